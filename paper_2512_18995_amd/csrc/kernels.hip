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

// Compile-time loop: every index is a constant expression, so register
// arrays indexed by it stay in VGPRs.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}
#define DQ_SF(N, ...) static_for<0, (N)>([&](auto ic_) { constexpr int i = decltype(ic_)::value; __VA_ARGS__; })

// Read-only tables (op lists, gate matrices) are read through the constant
// address space so that wave-uniform reads become scalar loads.
template <typename T> using cptr = __attribute__((address_space(4))) const T *;
template <typename T> __device__ __forceinline__ cptr<T> to_const(const T *p) { return (cptr<T>)(uintptr_t)p; }
template <typename V> __device__ __forceinline__ V ldc(cptr<V> p, int k) { return V{p[k].x, p[k].y}; }
__device__ __forceinline__ TOp ld_op(cptr<TOp> ops, int k) {
    const cptr<int32_t> w = (cptr<int32_t>)(ops + k);
    TOp o;
    o.kind = w[0];
    o.q0 = w[1];
    o.q1 = w[2];
    o.gen = w[3];
    o.slot = w[4];
    o.lslot = w[5];
    return o;
}

// Amplitudes are a plain aligned pair (not HIP's union-based float2/double2,
// which keeps register arrays of it from being promoted to VGPRs).
template <typename T> struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};
template <typename T> using cx = cpx<T>;
using C64 = cpx<float>;
using C128 = cpx<double>;

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * b + c
template <typename V> __device__ __forceinline__ V cmac(V a, V b, V c) {
    return V{fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
template <typename V> __device__ __forceinline__ V cneg(V a) { return V{-a.x, -a.y}; }
// component-wise select (a struct-valued ?: becomes a pointer select plus a
// copy through memory, which keeps register arrays out of VGPRs)
template <typename V> __device__ __forceinline__ V csel(bool c, V a, V b) { return V{c ? a.x : b.x, c ? a.y : b.y}; }

template <typename V> __device__ __forceinline__ V shfl_xor_c(V a, int mask) {
    return V{__shfl_xor(a.x, mask), __shfl_xor(a.y, mask)};
}

__device__ __forceinline__ int64_t insert_zero(int64_t x, int b) {
    return ((x >> b) << (b + 1)) | (x & ((int64_t(1) << b) - 1));
}

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

template <typename T>
__global__ void k_prepare(const DGate *gates, const double2 *fixed, const DSlot *slots, int nslots,
                          const double *params, int64_t pstride, const double *data, int64_t dstride,
                          cx<T> *mats, int64_t block) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (s >= nslots) return;
    const DSlot sl = slots[s];
    cx<T> *out = mats + b * block + sl.off;
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
        if (g.src == SRC_PARAM) v = params[b * pstride + g.idx];
        else if (g.src == SRC_DATA) v = data[b * dstride + g.idx];
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
template <typename T>
__global__ __launch_bounds__(256) void k_init_product(cx<T> *st, int n, const cx<T> *mats, int64_t mstride,
                                                      const int64_t *fold_off) {
    __shared__ double2 u[64][2];
    const int64_t b = blockIdx.y;
    if (threadIdx.x < n) {
        const int64_t off = fold_off[threadIdx.x];
        if (off < 0) {
            u[threadIdx.x][0] = double2{1.0, 0.0};
            u[threadIdx.x][1] = double2{0.0, 0.0};
        } else {
            const cx<T> *m = mats + b * mstride + off;
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

// ============================================================ plain per-gate sweeps
template <typename T>
__global__ __launch_bounds__(256) void k_gate1(cx<T> *st, int n, int64_t total, int bit, const cx<T> *mats,
                                               int64_t mstride, int64_t off) {
    const int64_t halfmask = (int64_t(1) << (n - 1)) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i >> (n - 1), k = i & halfmask;
        const int64_t j0 = insert_zero(k, bit), j1 = j0 | (int64_t(1) << bit);
        const cx<T> *m = mats + b * mstride + off;
        cx<T> *p = st + (b << n);
        const cx<T> a0 = p[j0], a1 = p[j1];
        p[j0] = cmac(m[0], a0, cmul(m[1], a1));
        p[j1] = cmac(m[2], a0, cmul(m[3], a1));
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

// ============================================================ register tiles
// Tile-local index u = (register index i) << 6 | lane.  Bit q of u: lane bit
// for q < 6, register bit q-6 otherwise.
__device__ __forceinline__ bool tbit(int i, int lane, int q) {
    return ((((unsigned)i << 6) | (unsigned)lane) >> q) & 1u;
}

template <int K> struct Pair {   // the i-th index pair (i0, i1) differing in register bit K
    static constexpr int lo(int i) { return ((i >> K) << (K + 1)) | (i & ((1 << K) - 1)); }
    static constexpr int hi(int i) { return lo(i) | (1 << K); }
};

template <typename V, int NR, int K>
__device__ __forceinline__ void reg_1q(V (&v)[NR], V m00, V m01, V m10, V m11) {
    DQ_SF(NR / 2, {
        constexpr int i0 = Pair<K>::lo(i), i1 = Pair<K>::hi(i);
        const V a0 = v[i0], a1 = v[i1];
        v[i0] = cmac(m00, a0, cmul(m01, a1));
        v[i1] = cmac(m10, a0, cmul(m11, a1));
    });
}

template <typename V, int NR, int K>
__device__ __forceinline__ void reg_cnot(V (&v)[NR], int cq, int lane) {
    DQ_SF(NR / 2, {
        constexpr int i0 = Pair<K>::lo(i), i1 = Pair<K>::hi(i);
        const bool c = tbit(i0, lane, cq);
        const V a0 = v[i0], a1 = v[i1];
        v[i0] = csel(c, a1, a0);
        v[i1] = csel(c, a0, a1);
    });
}

// swap of two register bits K1 < K2
template <typename V, int NR, int K1, int K2>
__device__ __forceinline__ void reg_swap(V (&v)[NR]) {
    DQ_SF(NR, {
        if constexpr (((i >> K1) & 1) && !((i >> K2) & 1)) {
            constexpr int j = i ^ (1 << K1) ^ (1 << K2);
            const V t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    });
}

// swap of lane bit l with register bit K
template <typename V, int NR, int K>
__device__ __forceinline__ void lane_reg_swap(V (&v)[NR], int l, int lane) {
    const bool hl = (lane >> l) & 1;
    DQ_SF(NR / 2, {
        constexpr int i0 = Pair<K>::lo(i), i1 = Pair<K>::hi(i);
        const V o0 = shfl_xor_c(v[i1], 1 << l), o1 = shfl_xor_c(v[i0], 1 << l);
        v[i0] = csel(hl, o0, v[i0]);
        v[i1] = csel(hl, v[i1], o1);
    });
}

template <typename T, typename V, int NR, int K>
__device__ __forceinline__ T reg_xy_sum(const V (&v)[NR], const V (&l)[NR], bool isY) {
    T s = 0;
    DQ_SF(NR, {
        V o = v[i ^ (1 << K)];
        if (isY) o = csel(((i >> K) & 1) != 0, V{-o.y, o.x}, V{o.y, -o.x});   // (Yv)_1 = i v_0, (Yv)_0 = -i v_1
        s += l[i].x * o.y - l[i].y * o.x;
    });
    return s;
}

#define DQ_REG_DISPATCH(k, NR, CALL)                                          \
    switch (k) {                                                              \
    case 0: if constexpr (NR > 1) { constexpr int K_ = 0; CALL; } break;      \
    case 1: if constexpr (NR > 2) { constexpr int K_ = 1; CALL; } break;      \
    case 2: if constexpr (NR > 4) { constexpr int K_ = 2; CALL; } break;      \
    case 3: if constexpr (NR > 8) { constexpr int K_ = 3; CALL; } break;      \
    case 4: if constexpr (NR > 16) { constexpr int K_ = 4; CALL; } break;     \
    case 5: if constexpr (NR > 32) { constexpr int K_ = 5; CALL; } break;     \
    default: break;                                                           \
    }

template <typename V, int NR, int K1>
__device__ __forceinline__ void reg_swap_k2(V (&v)[NR], int k2) {
    switch (k2) {
    case 1: if constexpr (NR > 2 && K1 < 1) reg_swap<V, NR, K1, 1>(v); break;
    case 2: if constexpr (NR > 4 && K1 < 2) reg_swap<V, NR, K1, 2>(v); break;
    case 3: if constexpr (NR > 8 && K1 < 3) reg_swap<V, NR, K1, 3>(v); break;
    case 4: if constexpr (NR > 16 && K1 < 4) reg_swap<V, NR, K1, 4>(v); break;
    case 5: if constexpr (NR > 32 && K1 < 5) reg_swap<V, NR, K1, 5>(v); break;
    default: break;
    }
}

template <typename T, int NR>
__device__ __forceinline__ void apply_op(cx<T> (&v)[NR], const TOp &op, cptr<cx<T>> m, int lane) {
    using V = cx<T>;
    switch (op.kind) {
    case TK_1Q: {
        const V m00 = ldc(m, op.slot), m01 = ldc(m, op.slot + 1), m10 = ldc(m, op.slot + 2), m11 = ldc(m, op.slot + 3);
        if (op.q0 < 6) {
            const bool hi = (lane >> op.q0) & 1;
            const V cs = csel(hi, m11, m00), co = csel(hi, m10, m01);
            DQ_SF(NR, { v[i] = cmac(cs, v[i], cmul(co, shfl_xor_c(v[i], 1 << op.q0))); });
        } else {
            DQ_REG_DISPATCH(op.q0 - 6, NR, (reg_1q<V, NR, K_>(v, m00, m01, m10, m11)));
        }
        break;
    }
    case TK_1QDIAG: {
        const V d0 = ldc(m, op.slot), d1 = ldc(m, op.slot + 3);
        DQ_SF(NR, { v[i] = cmul(csel(tbit(i, lane, op.q0), d1, d0), v[i]); });
        break;
    }
    case TK_CNOT: {
        if (op.q1 < 6) {
            DQ_SF(NR, {
                const V o = shfl_xor_c(v[i], 1 << op.q1);
                v[i] = csel(tbit(i, lane, op.q0), o, v[i]);
            });
        } else {
            DQ_REG_DISPATCH(op.q1 - 6, NR, (reg_cnot<V, NR, K_>(v, op.q0, lane)));
        }
        break;
    }
    case TK_CZ: {
        DQ_SF(NR, { v[i] = csel(tbit(i, lane, op.q0) && tbit(i, lane, op.q1), cneg(v[i]), v[i]); });
        break;
    }
    case TK_2QDIAG: {
        const V d0 = ldc(m, op.slot), d1 = ldc(m, op.slot + 5), d2 = ldc(m, op.slot + 10), d3 = ldc(m, op.slot + 15);
        DQ_SF(NR, {
            const bool a = tbit(i, lane, op.q0), b = tbit(i, lane, op.q1);
            v[i] = cmul(csel(a, csel(b, d3, d2), csel(b, d1, d0)), v[i]);
        });
        break;
    }
    case TK_SWAP: {
        const int a = op.q0 < op.q1 ? op.q0 : op.q1, b = op.q0 < op.q1 ? op.q1 : op.q0;
        if (b < 6) {
            const int mask = (1 << a) | (1 << b);
            const bool differ = ((lane >> a) ^ (lane >> b)) & 1;
            DQ_SF(NR, {
                const V o = shfl_xor_c(v[i], mask);
                v[i] = csel(differ, o, v[i]);
            });
        } else if (a < 6) {
            DQ_REG_DISPATCH(b - 6, NR, (lane_reg_swap<V, NR, K_>(v, a, lane)));
        } else {
            DQ_REG_DISPATCH(a - 6, NR, (reg_swap_k2<V, NR, K_>(v, b - 6)));
        }
        break;
    }
    default: break;
    }
}

// sum over this lane's register amplitudes of Im(conj(l) * (G v))
template <typename T, int NR>
__device__ __forceinline__ T gen_local(const cx<T> (&v)[NR], const cx<T> (&l)[NR], const TOp &op, int lane) {
    using V = cx<T>;
    T s = 0;
    switch (op.gen) {
    case GEN_Z:
        DQ_SF(NR, {
            const T t = l[i].x * v[i].y - l[i].y * v[i].x;
            s += tbit(i, lane, op.q0) ? -t : t;
        });
        break;
    case GEN_ZZ:
        DQ_SF(NR, {
            const T t = l[i].x * v[i].y - l[i].y * v[i].x;
            s += (tbit(i, lane, op.q0) != tbit(i, lane, op.q1)) ? -t : t;
        });
        break;
    case GEN_P11:
        DQ_SF(NR, {
            const T t = l[i].x * v[i].y - l[i].y * v[i].x;
            s += (tbit(i, lane, op.q0) && tbit(i, lane, op.q1)) ? t : T(0);
        });
        break;
    case GEN_X:
    case GEN_Y: {
        const bool isY = op.gen == GEN_Y;
        if (op.q0 < 6) {
            DQ_SF(NR, {
                V o = shfl_xor_c(v[i], 1 << op.q0);
                if (isY) o = csel(((lane >> op.q0) & 1) != 0, V{-o.y, o.x}, V{o.y, -o.x});
                s += l[i].x * o.y - l[i].y * o.x;
            });
        } else {
            DQ_REG_DISPATCH(op.q0 - 6, NR, (s = reg_xy_sum<T, V, NR, K_>(v, l, isY)));
        }
        break;
    }
    default: break;
    }
    return s;
}

template <int R>
__device__ __forceinline__ int64_t tile_base(int64_t t, const int32_t *rb) {
    int64_t base = t << 6;
#pragma unroll
    for (int k = 0; k < R; ++k) base = insert_zero(base, rb[k]);
    return base;
}

template <int R>
__device__ __forceinline__ int64_t reg_off(int i, const int32_t *rb) {
    int64_t o = 0;
#pragma unroll
    for (int k = 0; k < R; ++k)
        if ((i >> k) & 1) o += int64_t(1) << rb[k];
    return o;
}

template <typename T, int R>
__global__ __launch_bounds__(64) void k_tile_fwd(TileArgs a) {
    using V = cx<T>;
    constexpr int NR = 1 << R;
    const int lane = threadIdx.x;
    const int tshift = a.n - 6 - R;
    const int64_t total = a.batch << tshift;
    const int64_t tmask = (int64_t(1) << tshift) - 1;
    const cptr<TOp> ops = to_const(a.ops);
    V v[NR];
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int64_t b = tile >> tshift;
        V *tp = (V *)a.st + (b << a.n) + tile_base<R>(tile & tmask, a.rbits);   // wave-uniform
        const cptr<V> m = to_const((const V *)a.mats + b * a.mstride);
        DQ_SF(NR, { v[i] = (tp + reg_off<R>(i, a.rbits))[lane]; });
        for (int k = 0; k < a.nops; ++k) {
            const TOp op = ld_op(ops, k);
            apply_op<T, NR>(v, op, m, lane);
        }
        DQ_SF(NR, { (tp + reg_off<R>(i, a.rbits))[lane] = v[i]; });
    }
}

template <typename T, int R>
__global__ __launch_bounds__(64) void k_tile_adj(TileArgs a) {
    using V = cx<T>;
    constexpr int NR = 1 << R;
    extern __shared__ double acc[];   // [nlslots][64], one entry per lane
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.y;
    const int w = blockIdx.x;
    const int tshift = a.n - 6 - R;
    const int64_t tps = int64_t(1) << tshift;
    const cptr<TOp> ops = to_const(a.ops);
    const cptr<V> m = to_const((const V *)a.mats + b * a.mstride);
    for (int s = 0; s < a.nlslots; ++s) acc[s * 64 + lane] = 0.0;
    V v[NR], l[NR];
    for (int64_t t = w; t < tps; t += a.wps) {
        const int64_t base = (b << a.n) + tile_base<R>(t, a.rbits);   // wave-uniform
        V *pp = (V *)a.st + base;
        V *qp = (V *)a.lam + base;
        DQ_SF(NR, {
            v[i] = (pp + reg_off<R>(i, a.rbits))[lane];
            l[i] = (qp + reg_off<R>(i, a.rbits))[lane];
        });
        for (int k = 0; k < a.nops; ++k) {
            const TOp op = ld_op(ops, k);
            if (op.lslot >= 0) acc[op.lslot * 64 + lane] += (double)gen_local<T, NR>(v, l, op, lane);
            apply_op<T, NR>(v, op, m, lane);
            apply_op<T, NR>(l, op, m, lane);
        }
        DQ_SF(NR, {
            (pp + reg_off<R>(i, a.rbits))[lane] = v[i];
            (qp + reg_off<R>(i, a.rbits))[lane] = l[i];
        });
    }
    for (int s = 0; s < a.nlslots; ++s) {
        double x = acc[s * 64 + lane];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) a.partial[(b * a.wps + w) * (int64_t)a.ngrad + a.lslot_gslot[s]] = x;
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

constexpr int EXP_TM = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_expval_part(const cx<T> *st, int n, const DGroup *groups, int ngroups,
                                                     const DTerm *terms, int nterms, double *partial, int eb) {
    __shared__ double red[4][2 * EXP_TM];
    const int64_t b = blockIdx.y;
    const int64_t N = int64_t(1) << n;
    const cx<T> *p = st + b * N;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int g = 0; g < ngroups; ++g) {
        const DGroup G = groups[g];
        for (int c0 = G.t0; c0 < G.t1; c0 += EXP_TM) {
            const int nt = (G.t1 - c0) < EXP_TM ? (G.t1 - c0) : EXP_TM;
            uint64_t z[EXP_TM];
            double ar[EXP_TM], ai[EXP_TM];
#pragma unroll
            for (int t = 0; t < EXP_TM; ++t) {
                z[t] = t < nt ? terms[c0 + t].zmask : 0;
                ar[t] = 0.0;
                ai[t] = 0.0;
            }
            for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
                 j += (int64_t)eb * blockDim.x) {
                const cx<T> a = p[j], o = p[j ^ (int64_t)G.xmask];
                const double pr = (double)(o.x * a.x + o.y * a.y), pi = (double)(o.x * a.y - o.y * a.x);
#pragma unroll
                for (int t = 0; t < EXP_TM; ++t) {
                    if (t < nt) {
                        const bool neg = __popcll((uint64_t)j & z[t]) & 1;
                        ar[t] += neg ? -pr : pr;
                        ai[t] += neg ? -pi : pi;
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < EXP_TM; ++t) {
                if (t < nt) {
                    const double xr = wave_sum(ar[t]), xi = wave_sum(ai[t]);
                    if (lane == 0) {
                        red[wv][2 * t] = xr;
                        red[wv][2 * t + 1] = xi;
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x < 2 * nt) {
                const double s = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
                partial[((b * eb + blockIdx.x) * (int64_t)nterms + c0) * 2 + threadIdx.x] = s;
            }
            __syncthreads();
        }
    }
}

__global__ void k_expval_final(const double *partial, int64_t batch, int eb, const DTerm *terms, int nterms,
                               int nobs, double *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= batch * nobs) return;
    const int64_t b = i / nobs;
    const int o = (int)(i % nobs);
    double e = 0.0;
    for (int t = 0; t < nterms; ++t) {
        const DTerm tm = terms[t];
        if (tm.obs != o) continue;
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < eb; ++k) {
            sr += partial[((b * eb + k) * (int64_t)nterms + t) * 2];
            si += partial[((b * eb + k) * (int64_t)nterms + t) * 2 + 1];
        }
        e += tm.wr * sr - tm.wi * si;
    }
    out[i] = e;
}

// lambda_j = sum_k gout[b, obs_k] * coef_k i^{nY_k} (-1)^{|(j^x_k) & z_k|} psi_{j ^ x_k}
template <typename T>
__global__ __launch_bounds__(256) void k_lambda(const cx<T> *psi, cx<T> *lam, int n, int64_t total, const DGroup *groups,
                                                int ngroups, const DTerm *terms, const double *gout, int nobs) {
    const int64_t mask = (int64_t(1) << n) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i >> n, j = i & mask;
        const cx<T> *p = psi + (b << n);
        double ar = 0.0, ai = 0.0;
        for (int g = 0; g < ngroups; ++g) {
            const DGroup G = groups[g];
            const int64_t jx = j ^ (int64_t)G.xmask;
            const cx<T> o = p[jx];
            const double ox = (double)o.x, oy = (double)o.y;
            for (int t = G.t0; t < G.t1; ++t) {
                const DTerm tm = terms[t];
                const double go = gout[b * nobs + tm.obs];
                const double cr = go * tm.wr, ci = go * tm.wi;
                double tr = cr * ox - ci * oy, ti = cr * oy + ci * ox;
                if (__popcll((uint64_t)jx & tm.zmask) & 1) {
                    tr = -tr;
                    ti = -ti;
                }
                ar += tr;
                ai += ti;
            }
        }
        lam[i] = cx<T>{(T)ar, (T)ai};
    }
}

}  // namespace

// ============================================================ launchers
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

hipError_t launch_init_product(int dbl, void *st, int32_t n, int64_t batch, const void *mats, int64_t mstride,
                               const int64_t *fold_off, hipStream_t s) {
    const int64_t N = int64_t(1) << n;
    dim3 grid(grid_for(N, 256, 8192), (unsigned)batch);
    if (dbl)
        hipLaunchKernelGGL(k_init_product<double>, grid, dim3(256), 0, s, (C128 *)st, n, (const C128 *)mats,
                           mstride, fold_off);
    else
        hipLaunchKernelGGL(k_init_product<float>, grid, dim3(256), 0, s, (C64 *)st, n, (const C64 *)mats,
                           mstride, fold_off);
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

// Resident single-wave workgroups of a tile kernel on the current device
// (occupancy x compute units), cached per device and instantiation.
template <typename K>
static int resident_waves(K kernel, size_t lds, int key) {
    static int cache[64][32];
    static bool init = false;
    if (!init) {
        for (auto &r : cache)
            for (int &c : r) c = 0;
        init = true;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev >= 64) dev = 0;
    int &c = cache[dev][key & 31];
    if (c == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, lds) != hipSuccess || per_cu < 1)
            per_cu = 2;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        c = per_cu * cus;
    }
    return c;
}

static unsigned tile_grid(int64_t tiles, int resident) {
    // one resident wave per slot; each wave walks a strided subset of the tiles
    const int64_t cap = resident > 0 ? resident : 4096;
    return (unsigned)(tiles < cap ? (tiles < 1 ? 1 : tiles) : cap);
}

template <typename T, int R>
static void tile_fwd_r(const TileArgs &a, hipStream_t s) {
    const int key = (sizeof(T) == 8 ? 16 : 0) + R;
    const unsigned g = tile_grid(a.batch << (a.n - 6 - R), resident_waves(k_tile_fwd<T, R>, 0, key));
    hipLaunchKernelGGL((k_tile_fwd<T, R>), dim3(g), dim3(64), 0, s, a);
}

template <typename T>
static void tile_fwd_t(const TileArgs &a, hipStream_t s) {
    switch (a.R) {
    case 1: tile_fwd_r<T, 1>(a, s); break;
    case 2: tile_fwd_r<T, 2>(a, s); break;
    case 3: tile_fwd_r<T, 3>(a, s); break;
    case 4: tile_fwd_r<T, 4>(a, s); break;
    case 5: tile_fwd_r<T, 5>(a, s); break;
    default:
        if constexpr (sizeof(T) == 4) tile_fwd_r<T, 6>(a, s);
        break;
    }
}

hipError_t launch_tile_fwd(int dbl, const TileArgs &a, hipStream_t s) {
    if (dbl) {
        if (a.R > 5) return hipErrorInvalidValue;
        tile_fwd_t<double>(a, s);
    } else {
        tile_fwd_t<float>(a, s);
    }
    DQ_LAUNCH_RET;
}

template <typename T>
static void tile_adj_t(const TileArgs &a, hipStream_t s) {
    dim3 g((unsigned)a.wps, (unsigned)a.batch);
    const size_t lds = sizeof(double) * 64 * (a.nlslots > 0 ? a.nlslots : 1);
    switch (a.R) {
    case 1: hipLaunchKernelGGL((k_tile_adj<T, 1>), g, dim3(64), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_tile_adj<T, 2>), g, dim3(64), lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_tile_adj<T, 3>), g, dim3(64), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_tile_adj<T, 4>), g, dim3(64), lds, s, a); break;
    default:
        if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_tile_adj<T, 5>), g, dim3(64), lds, s, a);
        break;
    }
}

int tile_adj_capacity(int dbl, int R) {
    const size_t lds = sizeof(double) * 64 * 32;     // the most accumulator slots a pass may use
    const int key = 8 + (dbl ? 16 : 0) + R;
    if (dbl) {
        switch (R) {
        case 1: return resident_waves(k_tile_adj<double, 1>, lds, key);
        case 2: return resident_waves(k_tile_adj<double, 2>, lds, key);
        case 3: return resident_waves(k_tile_adj<double, 3>, lds, key);
        default: return resident_waves(k_tile_adj<double, 4>, lds, key);
        }
    }
    switch (R) {
    case 1: return resident_waves(k_tile_adj<float, 1>, lds, key);
    case 2: return resident_waves(k_tile_adj<float, 2>, lds, key);
    case 3: return resident_waves(k_tile_adj<float, 3>, lds, key);
    case 4: return resident_waves(k_tile_adj<float, 4>, lds, key);
    default: return resident_waves(k_tile_adj<float, 5>, lds, key);
    }
}

hipError_t launch_tile_adj(int dbl, const TileArgs &a, hipStream_t s) {
    if (a.nlslots > MAX_LSLOTS) return hipErrorInvalidValue;
    if (dbl) {
        if (a.R > 4) return hipErrorInvalidValue;
        tile_adj_t<double>(a, s);
    } else {
        if (a.R > 5) return hipErrorInvalidValue;
        tile_adj_t<float>(a, s);
    }
    DQ_LAUNCH_RET;
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

hipError_t launch_expval(int dbl, const void *st, int32_t n, int64_t batch, const DGroup *groups, int32_t ngroups,
                         const DTerm *terms, int32_t nterms, int32_t nobs, double *partial, int32_t eb, double *out,
                         hipStream_t s) {
    dim3 g((unsigned)eb, (unsigned)batch);
    if (dbl)
        hipLaunchKernelGGL(k_expval_part<double>, g, dim3(256), 0, s, (const C128 *)st, n, groups, ngroups, terms,
                           nterms, partial, eb);
    else
        hipLaunchKernelGGL(k_expval_part<float>, g, dim3(256), 0, s, (const C64 *)st, n, groups, ngroups, terms,
                           nterms, partial, eb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = batch * nobs;
    hipLaunchKernelGGL(k_expval_final, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s, partial, batch, eb,
                       terms, nterms, nobs, out);
    DQ_LAUNCH_RET;
}

hipError_t launch_lambda(int dbl, const void *psi, void *lam, int32_t n, int64_t batch, const DGroup *groups,
                         int32_t ngroups, const DTerm *terms, const double *grad_out, int32_t nobs, hipStream_t s) {
    const int64_t total = batch << n;
    if (dbl)
        hipLaunchKernelGGL(k_lambda<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, (const C128 *)psi,
                           (C128 *)lam, n, total, groups, ngroups, terms, grad_out, nobs);
    else
        hipLaunchKernelGGL(k_lambda<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, (const C64 *)psi,
                           (C64 *)lam, n, total, groups, ngroups, terms, grad_out, nobs);
    DQ_LAUNCH_RET;
}

}  // namespace dq
