// tile_dev.h -- register-tile device code of libdq, shared by the library's
// kernels (kernels.hip) and by the passes it compiles at plan time (the
// runtime hands this header to hipRTC), so both use one layout of the tile
// argument block and one implementation of every operation.
//
// A tile is 2^(6+R) amplitudes owned by one wave64: lane bits 0..2 are
// physical bits 0..2 (eight consecutive amplitudes per lane group), lane bits
// 3..5 and the R register bits are physical bits chosen per pass.
#pragma once
#include <stdint.h>
#include <type_traits>

namespace dq {

// Generator of a differentiable gate, as seen by the adjoint sweep:
//   GEN_X/Y/Z (one wire), GEN_ZZ (two wires) for exp(-i t G / 2)  -> dE/dt = Im<l|G|p>
//   GEN_P11 (|11><11| on two wires) for CP(t) = exp(i t P11)         -> dE/dt = -2 Im<l|P11|p>
enum : int32_t { GEN_NONE = 0, GEN_X = 1, GEN_Y = 2, GEN_Z = 3, GEN_ZZ = 4, GEN_P11 = 5 };

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
    int32_t nt;                // 1: loads and stores with the non-temporal hint
    int32_t pad_;
};


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
// The same, with a scheduling barrier after every 8 elements: loops that
// issue cross-lane shuffles would otherwise hoist all of them and hold every
// result in registers at once.
#define DQ_SF8(N, ...)                                                       \
    static_for<0, (N)>([&](auto ic_) {                                      \
        constexpr int i = decltype(ic_)::value;                             \
        __VA_ARGS__;                                                        \
        if constexpr ((i & 7) == 7) __builtin_amdgcn_sched_barrier(0);      \
    })

// Read-only tables (op lists, gate matrices) are read through the constant
// address space so that wave-uniform reads become scalar loads.
template <typename T> using cptr = __attribute__((address_space(4))) const T *;
template <typename T> __device__ __forceinline__ cptr<T> to_const(const T *p) { return (cptr<T>)(uintptr_t)p; }
template <typename V> __device__ __forceinline__ V ldc(cptr<V> p, int k) { return V{p[k].x, p[k].y}; }
// MultiEntry read field by field from the constant address space (scalar loads)

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

// Streaming accesses of tile passes: every amplitude is read once and written
// once per pass, so when the working set exceeds the last-level cache the
// loads and stores carry the non-temporal hint (a smaller state would stay in
// that cache between passes, and the hint costs it that reuse).
template <typename T> __device__ __forceinline__ cpx<T> ld_stream(const cpx<T> *p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 x = __builtin_nontemporal_load((const v2 *)p);
    return cpx<T>{x.x, x.y};
}
template <typename T> __device__ __forceinline__ void st_stream(cpx<T> *p, cpx<T> a) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 x;
    x.x = a.x;
    x.y = a.y;
    __builtin_nontemporal_store(x, (v2 *)p);
}

// Storage and arithmetic types of a tile may differ (complex64 states swept
// with float64 arithmetic): amplitudes are widened on load and rounded once
// on store.
template <typename T, typename S> __device__ __forceinline__ cpx<T> as_t(cpx<S> a) { return cpx<T>{(T)a.x, (T)a.y}; }

__device__ __forceinline__ float fm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fm(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * b + c
template <typename V> __device__ __forceinline__ V cmac(V a, V b, V c) {
    return V{fm(a.x, b.x, fm(-a.y, b.y, c.x)), fm(a.x, b.y, fm(a.y, b.x, c.y))};
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


// ============================================================ register tiles
// Tile-local index u = (register index i) << 6 | lane.  Bit q of u: lane bit
// for q < 6, register bit q-6 otherwise.

template <int K> struct Pair {   // the i-th index pair (i0, i1) differing in register bit K
    static constexpr int lo(int i) { return ((i >> K) << (K + 1)) | (i & ((1 << K) - 1)); }
    static constexpr int hi(int i) { return lo(i) | (1 << K); }
};

// The value held by the lane whose lane bit Q differs from this lane's.
// Bits 0..3 use DPP row patterns on the VALU: xor 1 and xor 2 are quad
// permutations, xor 4 is the half-row mirror (l -> l ^ 7) followed by the
// quad reversal (l -> l ^ 3), xor 8 the row mirror (l -> l ^ 15) followed by
// the half-row mirror.  Bit 4 uses the bitmask swizzle (xor 16 inside each
// 32-lane half), bit 5 a backwards permute.
template <int Q> __device__ __forceinline__ int lx_i(int a) {
    if constexpr (Q == 0) return __builtin_amdgcn_mov_dpp(a, 0xB1, 0xF, 0xF, false);
    else if constexpr (Q == 1) return __builtin_amdgcn_mov_dpp(a, 0x4E, 0xF, 0xF, false);
    else if constexpr (Q == 2)
        return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(a, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
    else if constexpr (Q == 3)
        return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(a, 0x140, 0xF, 0xF, false), 0x141, 0xF, 0xF, false);
    else if constexpr (Q == 4) return __builtin_amdgcn_ds_swizzle(a, 0x401F);
    else return __builtin_amdgcn_ds_bpermute((int)((threadIdx.x ^ 32u) << 2), a);
}
template <int Q> __device__ __forceinline__ float lx(float a) { return __int_as_float(lx_i<Q>(__float_as_int(a))); }
template <int Q> __device__ __forceinline__ double lx(double a) {
    const long long b = __double_as_longlong(a);
    const int lo = lx_i<Q>((int)(unsigned)(b & 0xffffffffll)), hi = lx_i<Q>((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int Q, typename V> __device__ __forceinline__ V lxc(V a) { return V{lx<Q>(a.x), lx<Q>(a.y)}; }

// Every op below updates NS state arrays of NR register amplitudes (NS = 1
// in the forward sweep, 2 = (psi, lambda) in the adjoint sweep), so that one
// dispatch serves both states and their arithmetic interleaves.  Template
// parameters K, C, A, B name register bits, Q lane bits: the operations are
// dispatched on where their qubits lie, so register selections, swaps and
// signs are resolved at compile time.
#define DQ_NS(...) static_for<0, NS>([&](auto sc_) { constexpr int s_ = decltype(sc_)::value; __VA_ARGS__; })

template <typename V, int NS, int NR, int K>
__device__ __forceinline__ void reg_1q(V (&v)[NS][NR], V m00, V m01, V m10, V m11) {
    DQ_SF(NR / 2, {
        constexpr int i0 = Pair<K>::lo(i), i1 = Pair<K>::hi(i);
        DQ_NS({
            const V a0 = v[s_][i0], a1 = v[s_][i1];
            v[s_][i0] = cmac(m00, a0, cmul(m01, a1));
            v[s_][i1] = cmac(m10, a0, cmul(m11, a1));
        });
    });
}

// real 2x2 (RY and products of RY, H, X, Z): 8 FMA per pair instead of 16
template <typename V, int NS, int NR, int K, typename T>
__device__ __forceinline__ void reg_1q_real(V (&v)[NS][NR], T m00, T m01, T m10, T m11) {
    DQ_SF(NR / 2, {
        constexpr int i0 = Pair<K>::lo(i), i1 = Pair<K>::hi(i);
        DQ_NS({
            const V a0 = v[s_][i0], a1 = v[s_][i1];
            v[s_][i0] = V{fm(m00, a0.x, m01 * a1.x), fm(m00, a0.y, m01 * a1.y)};
            v[s_][i1] = V{fm(m10, a0.x, m11 * a1.x), fm(m10, a0.y, m11 * a1.y)};
        });
    });
}

// [[c, i s], [i s, c]] (RX and its dagger): 8 FMA per pair
template <typename V, int NS, int NR, int K, typename T>
__device__ __forceinline__ void reg_1q_rx(V (&v)[NS][NR], T c, T s) {
    DQ_SF(NR / 2, {
        constexpr int i0 = Pair<K>::lo(i), i1 = Pair<K>::hi(i);
        DQ_NS({
            const V a0 = v[s_][i0], a1 = v[s_][i1];
            v[s_][i0] = V{fm(c, a0.x, -s * a1.y), fm(c, a0.y, s * a1.x)};
            v[s_][i1] = V{fm(c, a1.x, -s * a0.y), fm(c, a1.y, s * a0.x)};
        });
    });
}

template <typename V, int NS, int NR, int K>
__device__ __forceinline__ void reg_1q_diag(V (&v)[NS][NR], V d0, V d1) {
    DQ_SF(NR, { DQ_NS({ v[s_][i] = cmul(((i >> K) & 1) ? d1 : d0, v[s_][i]); }); });
}

// one-qubit gates on lane bit Q: this lane's own coefficient cs and its
// partner's co (chosen once per lane from the matrix row of its bit value)
template <typename V, int NS, int NR, int Q>
__device__ __forceinline__ void lane_1q(V (&v)[NS][NR], V cs, V co) {
    DQ_SF8(NR, { DQ_NS({ v[s_][i] = cmac(cs, v[s_][i], cmul(co, lxc<Q>(v[s_][i]))); }); });
}

template <typename V, int NS, int NR, int Q, typename T>
__device__ __forceinline__ void lane_1q_real(V (&v)[NS][NR], T cs, T co) {
    DQ_SF8(NR, {
        DQ_NS({
            const V o = lxc<Q>(v[s_][i]);
            v[s_][i] = V{fm(cs, v[s_][i].x, co * o.x), fm(cs, v[s_][i].y, co * o.y)};
        });
    });
}

template <typename V, int NS, int NR, int Q, typename T>
__device__ __forceinline__ void lane_1q_rx(V (&v)[NS][NR], T c, T sn) {
    DQ_SF8(NR, {
        DQ_NS({
            const V o = lxc<Q>(v[s_][i]);
            v[s_][i] = V{fm(c, v[s_][i].x, -sn * o.y), fm(c, v[s_][i].y, sn * o.x)};
        });
    });
}

// CNOT, target register bit K, control register bit C: a fixed exchange of
// register pairs
template <typename V, int NS, int NR, int K, int C>
__device__ __forceinline__ void reg_cnot_rr(V (&v)[NS][NR]) {
    if constexpr (K != C) DQ_SF(NR, {
        if constexpr (((i >> C) & 1) && !((i >> K) & 1)) {
            constexpr int j = i | (1 << K);
            DQ_NS({
                const V t = v[s_][i];
                v[s_][i] = v[s_][j];
                v[s_][j] = t;
            });
        }
    });
}

// CNOT, target register bit K, control lane bit (c = its value in this lane)
template <typename V, int NS, int NR, int K>
__device__ __forceinline__ void reg_cnot_lc(V (&v)[NS][NR], bool c) {
    DQ_SF(NR / 2, {
        constexpr int i0 = Pair<K>::lo(i), i1 = Pair<K>::hi(i);
        DQ_NS({
            const V a0 = v[s_][i0], a1 = v[s_][i1];
            v[s_][i0] = csel(c, a1, a0);
            v[s_][i1] = csel(c, a0, a1);
        });
    });
}

// CNOT, target lane bit Q, control register bit C: the registers whose bit C
// is set take their partner lane's value
template <typename V, int NS, int NR, int Q, int C>
__device__ __forceinline__ void lane_cnot_rc(V (&v)[NS][NR]) {
    DQ_SF8(NR, {
        if constexpr ((i >> C) & 1) { DQ_NS({ v[s_][i] = lxc<Q>(v[s_][i]); }); }
    });
}

// CNOT, target lane bit Q, control lane bit (c)
template <typename V, int NS, int NR, int Q>
__device__ __forceinline__ void lane_cnot_lc(V (&v)[NS][NR], bool c) {
    DQ_SF8(NR, {
        DQ_NS({
            const V o = lxc<Q>(v[s_][i]);
            v[s_][i] = csel(c, o, v[s_][i]);
        });
    });
}

// CZ on register bits A, B
template <typename V, int NS, int NR, int A, int B>
__device__ __forceinline__ void reg_cz_rr(V (&v)[NS][NR]) {
    if constexpr (A < B) DQ_SF(NR, {
        if constexpr (((i >> A) & 1) && ((i >> B) & 1)) { DQ_NS({ v[s_][i] = cneg(v[s_][i]); }); }
    });
}

// sign sg (+1 or -1, per lane) on the registers whose bit A is set
template <typename V, int NS, int NR, int A, typename T>
__device__ __forceinline__ void reg_sign(V (&v)[NS][NR], T sg) {
    DQ_SF(NR, {
        if constexpr ((i >> A) & 1) { DQ_NS({ v[s_][i] = V{sg * v[s_][i].x, sg * v[s_][i].y}; }); }
    });
}

template <int k, typename V> __device__ __forceinline__ V pick4(V d0, V d1, V d2, V d3) {
    if constexpr (k == 0) return d0;
    else if constexpr (k == 1) return d1;
    else if constexpr (k == 2) return d2;
    else return d3;
}

// two-qubit diagonal diag(d0, d1, d2, d3) over (bit A = msb, bit B), both
// register bits
template <typename V, int NS, int NR, int A, int B>
__device__ __forceinline__ void reg_2qdiag_rr(V (&v)[NS][NR], V d0, V d1, V d2, V d3) {
    if constexpr (A != B) DQ_SF(NR, {
        constexpr int k = 2 * ((i >> A) & 1) + ((i >> B) & 1);
        const V d = pick4<k>(d0, d1, d2, d3);
        DQ_NS({ v[s_][i] = cmul(d, v[s_][i]); });
    });
}

// diagonal factor e1 where register bit K is set, e0 elsewhere
template <typename V, int NS, int NR, int K>
__device__ __forceinline__ void reg_diag2(V (&v)[NS][NR], V e0, V e1) {
    DQ_SF(NR, { DQ_NS({ v[s_][i] = cmul(((i >> K) & 1) ? e1 : e0, v[s_][i]); }); });
}

// swap of two register bits K1 < K2
template <typename V, int NS, int NR, int K1, int K2>
__device__ __forceinline__ void reg_swap(V (&v)[NS][NR]) {
    if constexpr (K1 < K2) DQ_SF(NR, {
        if constexpr (((i >> K1) & 1) && !((i >> K2) & 1)) {
            constexpr int j = i ^ (1 << K1) ^ (1 << K2);
            DQ_NS({
                const V t = v[s_][i];
                v[s_][i] = v[s_][j];
                v[s_][j] = t;
            });
        }
    });
}

// swap of lane bit Q with register bit K
template <typename V, int NS, int NR, int K, int Q>
__device__ __forceinline__ void lane_reg_swap(V (&v)[NS][NR], int lane) {
    const bool hl = (lane >> Q) & 1;
    DQ_SF8(NR / 2, {
        constexpr int i0 = Pair<K>::lo(i), i1 = Pair<K>::hi(i);
        DQ_NS({
            const V o0 = lxc<Q>(v[s_][i1]), o1 = lxc<Q>(v[s_][i0]);
            v[s_][i0] = csel(hl, o0, v[s_][i0]);
            v[s_][i1] = csel(hl, v[s_][i1], o1);
        });
    });
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
// the same for a second register bit (name C_)
#define DQ_REG_DISPATCH_C(k, NR, CALL)                                        \
    switch (k) {                                                              \
    case 0: if constexpr (NR > 1) { constexpr int C_ = 0; CALL; } break;      \
    case 1: if constexpr (NR > 2) { constexpr int C_ = 1; CALL; } break;      \
    case 2: if constexpr (NR > 4) { constexpr int C_ = 2; CALL; } break;      \
    case 3: if constexpr (NR > 8) { constexpr int C_ = 3; CALL; } break;      \
    case 4: if constexpr (NR > 16) { constexpr int C_ = 4; CALL; } break;     \
    case 5: if constexpr (NR > 32) { constexpr int C_ = 5; CALL; } break;     \
    default: break;                                                           \
    }
#define DQ_LANE_DISPATCH(q, CALL)                                             \
    switch (q) {                                                              \
    case 0: { constexpr int Q_ = 0; CALL; } break;                            \
    case 1: { constexpr int Q_ = 1; CALL; } break;                            \
    case 2: { constexpr int Q_ = 2; CALL; } break;                            \
    case 3: { constexpr int Q_ = 3; CALL; } break;                            \
    case 4: { constexpr int Q_ = 4; CALL; } break;                            \
    case 5: { constexpr int Q_ = 5; CALL; } break;                            \
    default: break;                                                           \
    }

template <typename T, int NS, int NR>
__device__ __forceinline__ void apply_op(cx<T> (&v)[NS][NR], const TOp &op, cptr<cx<T>> m, int lane) {
    using V = cx<T>;
    switch (op.kind) {
    case TK_1Q: {
        const V m00 = ldc(m, op.slot), m01 = ldc(m, op.slot + 1), m10 = ldc(m, op.slot + 2), m11 = ldc(m, op.slot + 3);
        if (op.q0 < 6) {
            const bool hi = (lane >> op.q0) & 1;
            const V cs = csel(hi, m11, m00), co = csel(hi, m10, m01);
            DQ_LANE_DISPATCH(op.q0, (lane_1q<V, NS, NR, Q_>(v, cs, co)));
        } else {
            DQ_REG_DISPATCH(op.q0 - 6, NR, (reg_1q<V, NS, NR, K_>(v, m00, m01, m10, m11)));
        }
        break;
    }
    case TK_1QREAL: {
        const T m00 = m[op.slot].x, m01 = m[op.slot + 1].x, m10 = m[op.slot + 2].x, m11 = m[op.slot + 3].x;
        if (op.q0 < 6) {
            const bool hi = (lane >> op.q0) & 1;
            const T cs = hi ? m11 : m00, co = hi ? m10 : m01;
            DQ_LANE_DISPATCH(op.q0, (lane_1q_real<V, NS, NR, Q_, T>(v, cs, co)));
        } else {
            DQ_REG_DISPATCH(op.q0 - 6, NR, (reg_1q_real<V, NS, NR, K_, T>(v, m00, m01, m10, m11)));
        }
        break;
    }
    case TK_1QRX: {
        const T c = m[op.slot].x, sn = m[op.slot + 1].y;   // m01 = i s
        if (op.q0 < 6) {
            DQ_LANE_DISPATCH(op.q0, (lane_1q_rx<V, NS, NR, Q_, T>(v, c, sn)));
        } else {
            DQ_REG_DISPATCH(op.q0 - 6, NR, (reg_1q_rx<V, NS, NR, K_, T>(v, c, sn)));
        }
        break;
    }
    case TK_1QDIAG: {
        const V d0 = ldc(m, op.slot), d1 = ldc(m, op.slot + 3);
        if (op.q0 < 6) {
            const V d = csel(((lane >> op.q0) & 1) != 0, d1, d0);   // one factor per lane
            DQ_SF(NR, { DQ_NS({ v[s_][i] = cmul(d, v[s_][i]); }); });
        } else {
            DQ_REG_DISPATCH(op.q0 - 6, NR, (reg_1q_diag<V, NS, NR, K_>(v, d0, d1)));
        }
        break;
    }
    case TK_CNOT: {   // control q0, target q1
        if (op.q1 >= 6) {
            if (op.q0 >= 6) {
                DQ_REG_DISPATCH(op.q1 - 6, NR, DQ_REG_DISPATCH_C(op.q0 - 6, NR, (reg_cnot_rr<V, NS, NR, K_, C_>(v))));
            } else {
                const bool c = (lane >> op.q0) & 1;
                DQ_REG_DISPATCH(op.q1 - 6, NR, (reg_cnot_lc<V, NS, NR, K_>(v, c)));
            }
        } else {
            if (op.q0 >= 6) {
                DQ_LANE_DISPATCH(op.q1, DQ_REG_DISPATCH_C(op.q0 - 6, NR, (lane_cnot_rc<V, NS, NR, Q_, C_>(v))));
            } else {
                const bool c = (lane >> op.q0) & 1;
                DQ_LANE_DISPATCH(op.q1, (lane_cnot_lc<V, NS, NR, Q_>(v, c)));
            }
        }
        break;
    }
    case TK_CZ: {
        const int a = op.q0 < op.q1 ? op.q0 : op.q1, b = op.q0 < op.q1 ? op.q1 : op.q0;
        if (a >= 6) {
            DQ_REG_DISPATCH(a - 6, NR, DQ_REG_DISPATCH_C(b - 6, NR, (reg_cz_rr<V, NS, NR, K_, C_>(v))));
        } else if (b >= 6) {
            const T sg = ((lane >> a) & 1) ? T(-1) : T(1);
            DQ_REG_DISPATCH(b - 6, NR, (reg_sign<V, NS, NR, K_, T>(v, sg)));
        } else {
            const T sg = (((lane >> a) & (lane >> b)) & 1) ? T(-1) : T(1);
            DQ_SF(NR, { DQ_NS({ v[s_][i] = V{sg * v[s_][i].x, sg * v[s_][i].y}; }); });
        }
        break;
    }
    case TK_2QDIAG: {   // diag over (q0 = msb, q1)
        const V d0 = ldc(m, op.slot), d1 = ldc(m, op.slot + 5), d2 = ldc(m, op.slot + 10), d3 = ldc(m, op.slot + 15);
        if (op.q0 >= 6 && op.q1 >= 6) {
            DQ_REG_DISPATCH(op.q0 - 6, NR,
                            DQ_REG_DISPATCH_C(op.q1 - 6, NR, (reg_2qdiag_rr<V, NS, NR, K_, C_>(v, d0, d1, d2, d3))));
        } else if (op.q0 < 6 && op.q1 >= 6) {
            const bool a = (lane >> op.q0) & 1;
            const V e0 = csel(a, d2, d0), e1 = csel(a, d3, d1);
            DQ_REG_DISPATCH(op.q1 - 6, NR, (reg_diag2<V, NS, NR, K_>(v, e0, e1)));
        } else if (op.q0 >= 6) {
            const bool b = (lane >> op.q1) & 1;
            const V e0 = csel(b, d1, d0), e1 = csel(b, d3, d2);
            DQ_REG_DISPATCH(op.q0 - 6, NR, (reg_diag2<V, NS, NR, K_>(v, e0, e1)));
        } else {
            const bool a = (lane >> op.q0) & 1, b = (lane >> op.q1) & 1;
            const V d = csel(a, csel(b, d3, d2), csel(b, d1, d0));
            DQ_SF(NR, { DQ_NS({ v[s_][i] = cmul(d, v[s_][i]); }); });
        }
        break;
    }
    case TK_SWAP: {
        const int a = op.q0 < op.q1 ? op.q0 : op.q1, b = op.q0 < op.q1 ? op.q1 : op.q0;
        if (b < 6) {
            const int mask = (1 << a) | (1 << b);
            const bool differ = ((lane >> a) ^ (lane >> b)) & 1;
            DQ_SF8(NR, {
                DQ_NS({
                    const V o = shfl_xor_c(v[s_][i], mask);
                    v[s_][i] = csel(differ, o, v[s_][i]);
                });
            });
        } else if (a < 6) {
            DQ_REG_DISPATCH(b - 6, NR, DQ_LANE_DISPATCH(a, (lane_reg_swap<V, NS, NR, K_, Q_>(v, lane))));
        } else {
            DQ_REG_DISPATCH(a - 6, NR, DQ_REG_DISPATCH_C(b - 6, NR, (reg_swap<V, NS, NR, K_, C_>(v))));
        }
        break;
    }
    default: break;
    }
}

// Gradient terms: sums over this lane's registers of Im(conj(l) * (P v)) for
// the generator P of the op (t_i = Im(conj(l_i) v_i) for diagonal P).
template <typename T, typename V> __device__ __forceinline__ T im_dot(V l, V v) { return l.x * v.y - l.y * v.x; }

// sum of t_i with sign -1 where register bit K is set (A and B: where
// exactly one of them is set; P11: only where both are set)
template <typename T, typename V, int NR, int K>
__device__ __forceinline__ T reg_z_sum(const V (&v)[NR], const V (&l)[NR]) {
    T s = 0;
    DQ_SF(NR, {
        const T t = im_dot<T>(l[i], v[i]);
        if constexpr ((i >> K) & 1) s -= t;
        else s += t;
    });
    return s;
}
template <typename T, typename V, int NR, int A, int B>
__device__ __forceinline__ T reg_zz_sum(const V (&v)[NR], const V (&l)[NR]) {
    T s = 0;
    if constexpr (A < B) DQ_SF(NR, {
        const T t = im_dot<T>(l[i], v[i]);
        if constexpr (((i >> A) ^ (i >> B)) & 1) s -= t;
        else s += t;
    });
    return s;
}
template <typename T, typename V, int NR, int A, int B>
__device__ __forceinline__ T reg_p11_sum(const V (&v)[NR], const V (&l)[NR]) {
    T s = 0;
    if constexpr (A < B) DQ_SF(NR, {
        if constexpr ((i >> A) & (i >> B) & 1) s += im_dot<T>(l[i], v[i]);
    });
    return s;
}
template <typename T, typename V, int NR>
__device__ __forceinline__ T all_sum(const V (&v)[NR], const V (&l)[NR]) {
    T s = 0;
    DQ_SF(NR, { s += im_dot<T>(l[i], v[i]); });
    return s;
}
// sum of t_i over the registers whose bit K is set
template <typename T, typename V, int NR, int K>
__device__ __forceinline__ T reg_set_sum(const V (&v)[NR], const V (&l)[NR]) {
    T s = 0;
    DQ_SF(NR, {
        if constexpr ((i >> K) & 1) s += im_dot<T>(l[i], v[i]);
    });
    return s;
}

template <typename T, typename V, int NR, int K>
__device__ __forceinline__ T reg_xy_sum(const V (&v)[NR], const V (&l)[NR], bool isY) {
    T s = 0;
    DQ_SF(NR, {
        V o = v[i ^ (1 << K)];
        if (isY) {   // (Y v)_1 = i v_0, (Y v)_0 = -i v_1
            if constexpr ((i >> K) & 1) o = V{-o.y, o.x};
            else o = V{o.y, -o.x};
        }
        s += im_dot<T>(l[i], o);
    });
    return s;
}

template <typename T, typename V, int NR, int Q>
__device__ __forceinline__ T lane_xy_sum(const V (&v)[NR], const V (&l)[NR], bool isY, bool hi) {
    T s = 0;
    if (isY) {
        // (Y v) at this lane is -i p (bit 0) or +i p (bit 1) for the partner
        // value p, so Im(conj(l) (Y v)) = -+Re(conj(l) p): one sign per lane
        DQ_SF8(NR, {
            const V o = lxc<Q>(v[i]);
            s += l[i].x * o.x + l[i].y * o.y;
        });
        return hi ? s : -s;
    }
    DQ_SF8(NR, { s += im_dot<T>(l[i], lxc<Q>(v[i])); });
    return s;
}

template <typename T, int NR>
__device__ __forceinline__ T gen_local(const cx<T> (&v)[NR], const cx<T> (&l)[NR], const TOp &op, int lane) {
    using V = cx<T>;
    T s = 0;
    switch (op.gen) {
    case GEN_Z:
        if (op.q0 < 6) {
            s = all_sum<T, V, NR>(v, l);
            if ((lane >> op.q0) & 1) s = -s;
        } else {
            DQ_REG_DISPATCH(op.q0 - 6, NR, (s = reg_z_sum<T, V, NR, K_>(v, l)));
        }
        break;
    case GEN_ZZ: {
        const int a = op.q0 < op.q1 ? op.q0 : op.q1, b = op.q0 < op.q1 ? op.q1 : op.q0;
        if (a >= 6) {
            DQ_REG_DISPATCH(a - 6, NR, DQ_REG_DISPATCH_C(b - 6, NR, (s = reg_zz_sum<T, V, NR, K_, C_>(v, l))));
        } else if (b >= 6) {
            DQ_REG_DISPATCH(b - 6, NR, (s = reg_z_sum<T, V, NR, K_>(v, l)));
            if ((lane >> a) & 1) s = -s;
        } else {
            s = all_sum<T, V, NR>(v, l);
            if (((lane >> a) ^ (lane >> b)) & 1) s = -s;
        }
        break;
    }
    case GEN_P11: {
        const int a = op.q0 < op.q1 ? op.q0 : op.q1, b = op.q0 < op.q1 ? op.q1 : op.q0;
        if (a >= 6) {
            DQ_REG_DISPATCH(a - 6, NR, DQ_REG_DISPATCH_C(b - 6, NR, (s = reg_p11_sum<T, V, NR, K_, C_>(v, l))));
        } else if (b >= 6) {
            DQ_REG_DISPATCH(b - 6, NR, (s = reg_set_sum<T, V, NR, K_>(v, l)));
            if (!((lane >> a) & 1)) s = T(0);
        } else {
            s = all_sum<T, V, NR>(v, l);
            if (!((lane >> a) & (lane >> b) & 1)) s = T(0);
        }
        break;
    }
    case GEN_X:
    case GEN_Y: {
        const bool isY = op.gen == GEN_Y;
        if (op.q0 < 6) {
            const bool hi = (lane >> op.q0) & 1;
            DQ_LANE_DISPATCH(op.q0, (s = lane_xy_sum<T, V, NR, Q_>(v, l, isY, hi)));
        } else {
            DQ_REG_DISPATCH(op.q0 - 6, NR, (s = reg_xy_sum<T, V, NR, K_>(v, l, isY)));
        }
        break;
    }
    default: break;
    }
    return s;
}

// first amplitude of tile t: the tile index fills every physical bit that is
// not a tile bit (bits 0..2 and the 3 + R chosen bits are zero)
template <int R>
__device__ __forceinline__ int64_t tile_base(int64_t t, const int32_t *tb) {
    int64_t base = t << 3;
#pragma unroll
    for (int k = 0; k < R + 3; ++k) base = insert_zero(base, tb[k]);
    return base;
}

// this lane's offset inside a tile: lane bits 0..2 -> physical 0..2,
// lane bits 3..5 -> lbits[0..2]
__device__ __forceinline__ int64_t lane_off(int lane, const int32_t *lb) {
    int64_t o = lane & 7;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if ((lane >> (3 + k)) & 1) o += int64_t(1) << lb[k];
    return o;
}

template <int R>
__device__ __forceinline__ int64_t reg_off(int i, const int32_t *rb) {
    int64_t o = 0;
#pragma unroll
    for (int k = 0; k < R; ++k)
        if ((i >> k) & 1) o += int64_t(1) << rb[k];
    return o;
}

// occupancy target (waves per SIMD) of the register tiles: two for the
// largest tiles, more for small ones
template <typename T, int R> constexpr int tile_waves() { return (1 << R) * sizeof(T) >= 256 ? 1 : ((1 << R) * sizeof(T) >= 128 ? 2 : 3); }
// the adjoint holds two states per lane: two waves per SIMD up to 16
// complex64 (8 complex128) amplitudes per state
template <typename T, int R> constexpr int adj_waves() { return (1 << R) * sizeof(T) >= 128 ? 1 : ((1 << R) * sizeof(T) >= 64 ? 2 : 4); }

// One forward tile: load 2^R amplitudes per lane, run the operations
// (body(v): an op-list interpreter, or a pass compiled at plan time), store.
template <typename T, int R, typename S = T, typename Body>
__device__ __forceinline__ void fwd_tile(cx<S> *st, int64_t base, int64_t lo, const int32_t *rbits, bool nt,
                                         Body &&body) {
    using V = cx<T>;
    constexpr int NR = 1 << R;
    V v[1][NR];
    {
        cx<S> *tp = st + base;
        if (nt) {
            DQ_SF(NR, { v[0][i] = as_t<T>(ld_stream(tp + reg_off<R>(i, rbits) + lo)); });
        } else {
            DQ_SF(NR, { v[0][i] = as_t<T>((tp + reg_off<R>(i, rbits))[lo]); });
        }
    }
    body(v);
    // recompute the addresses for the stores rather than keeping the loads'
    // 2^R per-lane pointers alive across the operations
    asm volatile("" : "+s"(base));
    {
        cx<S> *tp = st + base;
        if (nt) {
            DQ_SF(NR, { st_stream(tp + reg_off<R>(i, rbits) + lo, as_t<S>(v[0][i])); });
        } else {
            DQ_SF(NR, { (tp + reg_off<R>(i, rbits))[lo] = as_t<S>(v[0][i]); });
        }
    }
}

// One adjoint work unit: tiles t = w, w + wps, ... of one sample, whose
// state starts at st + sbase and whose lambda starts at lam + lbase; body(v,
// acc) runs the pass on (psi, lambda), adding gradient terms into per-lane
// float64 accumulators in LDS, which are reduced over the wave into
// partial_row[lslot_gslot[s]].
template <typename T, int R, typename S = T, typename Body>
__device__ __forceinline__ void adj_unit(cx<S> *st, cx<S> *lam, int64_t sbase, int64_t lbase, int n,
                                         const int32_t *rbits, const int32_t *lbits, const int32_t *tbits, int nls,
                                         int64_t w, int64_t wps, double *partial_row, const int32_t *lslot_gslot,
                                         double *acc, int lane, bool nt, Body &&body) {
    using V = cx<T>;
    constexpr int NR = 1 << R;
    const int64_t tps = int64_t(1) << (n - 6 - R);
    for (int s = 0; s < nls; ++s) acc[s * 64 + lane] = 0.0;
    const int64_t lo = lane_off(lane, lbits);
    V v[2][NR];   // [0] = psi, [1] = lambda
    for (int64_t t = w; t < tps; t += wps) {
        int64_t base = tile_base<R>(t, tbits);   // wave-uniform
        {
            cx<S> *pp = st + sbase + base;
            cx<S> *qp = lam + lbase + base;
            if (nt) {
                DQ_SF(NR, {
                    v[0][i] = as_t<T>(ld_stream(pp + reg_off<R>(i, rbits) + lo));
                    v[1][i] = as_t<T>(ld_stream(qp + reg_off<R>(i, rbits) + lo));
                });
            } else {
                DQ_SF(NR, {
                    v[0][i] = as_t<T>((pp + reg_off<R>(i, rbits))[lo]);
                    v[1][i] = as_t<T>((qp + reg_off<R>(i, rbits))[lo]);
                });
            }
        }
        body(v, acc);
        asm volatile("" : "+s"(base));
        {
            cx<S> *pp = st + sbase + base;
            cx<S> *qp = lam + lbase + base;
            if (nt) {
                DQ_SF(NR, {
                    st_stream(pp + reg_off<R>(i, rbits) + lo, as_t<S>(v[0][i]));
                    st_stream(qp + reg_off<R>(i, rbits) + lo, as_t<S>(v[1][i]));
                });
            } else {
                DQ_SF(NR, {
                    (pp + reg_off<R>(i, rbits))[lo] = as_t<S>(v[0][i]);
                    (qp + reg_off<R>(i, rbits))[lo] = as_t<S>(v[1][i]);
                });
            }
        }
    }
    for (int s = 0; s < nls; ++s) {
        double x = acc[s * 64 + lane];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) partial_row[lslot_gslot[s]] = x;
    }
}

// ---------------------------------------------------------------- compiled passes
// The same operations with every operand position a compile-time constant:
// a pass compiled at plan time is a straight-line sequence of these calls
// (slots relative to the pass's first matrix), so register selections,
// swaps and CNOTs between register bits become renamings, and nothing is
// dispatched at run time.
template <typename T, int NS, int NR, int KIND, int Q0, int Q1, int SLOT>
__device__ __forceinline__ void op_s(cx<T> (&v)[NS][NR], cptr<cx<T>> m, int lane) {
    using V = cx<T>;
    if constexpr (KIND == TK_1Q) {
        const V m00 = ldc(m, SLOT), m01 = ldc(m, SLOT + 1), m10 = ldc(m, SLOT + 2), m11 = ldc(m, SLOT + 3);
        if constexpr (Q0 < 6) {
            const bool hi = (lane >> Q0) & 1;
            lane_1q<V, NS, NR, Q0>(v, csel(hi, m11, m00), csel(hi, m10, m01));
        } else {
            reg_1q<V, NS, NR, Q0 - 6>(v, m00, m01, m10, m11);
        }
    } else if constexpr (KIND == TK_1QREAL) {
        const T m00 = m[SLOT].x, m01 = m[SLOT + 1].x, m10 = m[SLOT + 2].x, m11 = m[SLOT + 3].x;
        if constexpr (Q0 < 6) {
            const bool hi = (lane >> Q0) & 1;
            lane_1q_real<V, NS, NR, Q0, T>(v, hi ? m11 : m00, hi ? m10 : m01);
        } else {
            reg_1q_real<V, NS, NR, Q0 - 6, T>(v, m00, m01, m10, m11);
        }
    } else if constexpr (KIND == TK_1QRX) {
        const T c = m[SLOT].x, sn = m[SLOT + 1].y;
        if constexpr (Q0 < 6) lane_1q_rx<V, NS, NR, Q0, T>(v, c, sn);
        else reg_1q_rx<V, NS, NR, Q0 - 6, T>(v, c, sn);
    } else if constexpr (KIND == TK_1QDIAG) {
        const V d0 = ldc(m, SLOT), d1 = ldc(m, SLOT + 3);
        if constexpr (Q0 < 6) {
            const V d = csel(((lane >> Q0) & 1) != 0, d1, d0);
            DQ_SF(NR, { DQ_NS({ v[s_][i] = cmul(d, v[s_][i]); }); });
        } else {
            reg_1q_diag<V, NS, NR, Q0 - 6>(v, d0, d1);
        }
    } else if constexpr (KIND == TK_CNOT) {   // control Q0, target Q1
        if constexpr (Q1 >= 6 && Q0 >= 6) reg_cnot_rr<V, NS, NR, Q1 - 6, Q0 - 6>(v);
        else if constexpr (Q1 >= 6) reg_cnot_lc<V, NS, NR, Q1 - 6>(v, (lane >> Q0) & 1);
        else if constexpr (Q0 >= 6) lane_cnot_rc<V, NS, NR, Q1, Q0 - 6>(v);
        else lane_cnot_lc<V, NS, NR, Q1>(v, (lane >> Q0) & 1);
    } else if constexpr (KIND == TK_CZ) {
        constexpr int A = Q0 < Q1 ? Q0 : Q1, B = Q0 < Q1 ? Q1 : Q0;
        if constexpr (A >= 6) {
            reg_cz_rr<V, NS, NR, A - 6, B - 6>(v);
        } else if constexpr (B >= 6) {
            reg_sign<V, NS, NR, B - 6, T>(v, ((lane >> A) & 1) ? T(-1) : T(1));
        } else {
            const T sg = (((lane >> A) & (lane >> B)) & 1) ? T(-1) : T(1);
            DQ_SF(NR, { DQ_NS({ v[s_][i] = V{sg * v[s_][i].x, sg * v[s_][i].y}; }); });
        }
    } else if constexpr (KIND == TK_2QDIAG) {   // diag over (Q0 = msb, Q1)
        const V d0 = ldc(m, SLOT), d1 = ldc(m, SLOT + 5), d2 = ldc(m, SLOT + 10), d3 = ldc(m, SLOT + 15);
        if constexpr (Q0 >= 6 && Q1 >= 6) {
            reg_2qdiag_rr<V, NS, NR, Q0 - 6, Q1 - 6>(v, d0, d1, d2, d3);
        } else if constexpr (Q1 >= 6) {
            const bool a = (lane >> Q0) & 1;
            reg_diag2<V, NS, NR, Q1 - 6>(v, csel(a, d2, d0), csel(a, d3, d1));
        } else if constexpr (Q0 >= 6) {
            const bool b = (lane >> Q1) & 1;
            reg_diag2<V, NS, NR, Q0 - 6>(v, csel(b, d1, d0), csel(b, d3, d2));
        } else {
            const bool a = (lane >> Q0) & 1, b = (lane >> Q1) & 1;
            const V d = csel(a, csel(b, d3, d2), csel(b, d1, d0));
            DQ_SF(NR, { DQ_NS({ v[s_][i] = cmul(d, v[s_][i]); }); });
        }
    } else if constexpr (KIND == TK_SWAP) {
        constexpr int A = Q0 < Q1 ? Q0 : Q1, B = Q0 < Q1 ? Q1 : Q0;
        if constexpr (B < 6) {
            const bool differ = ((lane >> A) ^ (lane >> B)) & 1;
            DQ_SF8(NR, {
                DQ_NS({
                    const V o = shfl_xor_c(v[s_][i], (1 << A) | (1 << B));
                    v[s_][i] = csel(differ, o, v[s_][i]);
                });
            });
        } else if constexpr (A < 6) {
            lane_reg_swap<V, NS, NR, B - 6, A>(v, lane);
        } else {
            reg_swap<V, NS, NR, A - 6, B - 6>(v);
        }
    }
}

// A run of consecutive one-qubit diagonal gates applied as one product
// diagonal.  Per lane the factor of amplitude (lane, register i) is fl times
// the product, over the run's register-bit gates j whose bit KS[j] is set in
// i, of r[j] = d1_j conj(d0_j) (fl already holds every d0_j and the lane-bit
// gates' factors; unitary diagonals have |d0| = 1).  The factors of the
// first (up to) three register bits are built as a product tree of at most
// eight values and applied in one multiply per amplitude; each further bit
// multiplies its ratio into the amplitudes where it is set.
//
// fl, r and the product tree are formed in double precision from the
// state-precision matrix entries and rounded once: a factor depends only on
// the lane's bits, so every amplitude that shares them (a 1/64 slice of the
// state) gets the same factor, and rounding errors of a single-precision
// product would add coherently over the whole slice (for a run of about 20
// gates, each of the 64 factors would carry about sqrt(20) roundings instead
// of one, the same error on millions of amplitudes).
template <int... KS> constexpr int pack_at(int j) {
    const int ks[] = {KS..., 0};
    return ks[j];
}
template <int... KS> constexpr int pack_compact(int i, int kt) {   // bit j = bit KS[j] of i, j < kt
    const int ks[] = {KS..., 0};
    int x = 0;
    for (int j = 0; j < kt; ++j)
        if ((i >> ks[j]) & 1) x |= 1 << j;
    return x;
}
template <int... KS> constexpr int pack_mask(int j) {   // bits of the first j entries
    const int ks[] = {KS..., 0};
    int mk = 0;
    for (int t = 0; t < j; ++t) mk |= 1 << ks[t];
    return mk;
}

template <typename T> __device__ __forceinline__ C128 widen(cx<T> a) { return C128{(double)a.x, (double)a.y}; }
template <typename T> __device__ __forceinline__ cx<T> narrow(C128 a) { return cx<T>{(T)a.x, (T)a.y}; }

template <typename T, int NS, int NR, int... KS>
__device__ __forceinline__ void diag_run(cx<T> (&v)[NS][NR], C128 fl, const C128 *r) {
    using V = cx<T>;
    constexpr int k = sizeof...(KS);
    constexpr int kt = k < 3 ? k : 3;              // bits covered by the factor table
    C128 fd[1 << kt];
    fd[0] = fl;
    static_for<0, kt>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        // f is indexed by the compacted bits of the table (bit j of the
        // index = register bit KS[j])
        static_for<0, (1 << j)>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            fd[i | (1 << j)] = cmul(fd[i], r[j]);
        });
    });
    V f[1 << kt];
    static_for<0, (1 << kt)>([&](auto ic) { f[decltype(ic)::value] = narrow<T>(fd[decltype(ic)::value]); });
    DQ_SF(NR, {
        constexpr int c = pack_compact<KS...>(i, kt);
        DQ_NS({ v[s_][i] = cmul(f[c], v[s_][i]); });
    });
    // the remaining register bits: their ratio on the amplitudes whose bit is set
    static_for<kt, k>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int kj = pack_at<KS...>(j);
        const V rj = narrow<T>(r[j]);
        DQ_SF(NR, {
            if constexpr ((i >> kj) & 1) { DQ_NS({ v[s_][i] = cmul(rj, v[s_][i]); }); }
        });
    });
}

// all of a run's gradient sums in one sweep over the registers: sa = sum
// t_i, sk[j] = sum t_i signed by register bit KS[j]
template <typename T, typename V, int NR, int... KS>
__device__ __forceinline__ void run_sums(const V (&v)[NR], const V (&l)[NR], T &sa, T *sk) {
    constexpr int k = sizeof...(KS);
    sa = 0;
    static_for<0, k>([&](auto jc) { sk[decltype(jc)::value] = 0; });
    DQ_SF(NR, {
        const T t = im_dot<T>(l[i], v[i]);
        sa += t;
        static_for<0, k>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr ((i >> pack_at<KS...>(j)) & 1) sk[j] -= t;
            else sk[j] += t;
        });
    });
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }

// Im<lambda| P |psi> summed over this lane's registers, for the generator P
// of a differentiable gate at compile-time positions
template <typename T, int NR, int GEN, int Q0, int Q1>
__device__ __forceinline__ T gen_s(const cx<T> (&v)[NR], const cx<T> (&l)[NR], int lane) {
    using V = cx<T>;
    if constexpr (GEN == GEN_Z) {
        if constexpr (Q0 < 6) {
            const T s = all_sum<T, V, NR>(v, l);
            return ((lane >> Q0) & 1) ? -s : s;
        } else {
            return reg_z_sum<T, V, NR, Q0 - 6>(v, l);
        }
    } else if constexpr (GEN == GEN_ZZ || GEN == GEN_P11) {
        constexpr int A = Q0 < Q1 ? Q0 : Q1, B = Q0 < Q1 ? Q1 : Q0;
        if constexpr (A >= 6) {
            if constexpr (GEN == GEN_ZZ) return reg_zz_sum<T, V, NR, A - 6, B - 6>(v, l);
            else return reg_p11_sum<T, V, NR, A - 6, B - 6>(v, l);
        } else if constexpr (B >= 6) {
            if constexpr (GEN == GEN_ZZ) {
                const T s = reg_z_sum<T, V, NR, B - 6>(v, l);
                return ((lane >> A) & 1) ? -s : s;
            } else {
                const T s = reg_set_sum<T, V, NR, B - 6>(v, l);
                return ((lane >> A) & 1) ? s : T(0);
            }
        } else {
            const T s = all_sum<T, V, NR>(v, l);
            if constexpr (GEN == GEN_ZZ) return (((lane >> A) ^ (lane >> B)) & 1) ? -s : s;
            else return (((lane >> A) & (lane >> B)) & 1) ? s : T(0);
        }
    } else if constexpr (GEN == GEN_X || GEN == GEN_Y) {
        if constexpr (Q0 < 6) return lane_xy_sum<T, V, NR, Q0>(v, l, GEN == GEN_Y, (lane >> Q0) & 1);
        else return reg_xy_sum<T, V, NR, Q0 - 6>(v, l, GEN == GEN_Y);
    } else {
        return T(0);
    }
}

// Kernel bodies of compiled passes.  The forward walks the tiles of every
// sample in a grid-stride loop; the adjoint runs work unit blockIdx.x of
// sample blockIdx.y (as the interpreted passes do).  a.mats points at the
// pass's first matrix.
template <typename T, int R, bool NT, typename S = T, typename Body>
__device__ __forceinline__ void jit_fwd(const TileArgs &a, Body &&body) {
    using V = cx<T>;
    const int lane = threadIdx.x;
    const int tshift = a.n - 6 - R;
    const int64_t total = a.batch << tshift;
    const int64_t tmask = (int64_t(1) << tshift) - 1;
    const int64_t lo = lane_off(lane, a.lbits);
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int64_t b = tile >> tshift;
        const int64_t base = (b << a.n) + tile_base<R>(tile & tmask, a.tbits);
        const cptr<V> m = to_const((const V *)a.mats + b * a.mstride);
        fwd_tile<T, R, S>((cx<S> *)a.st, base, lo, a.rbits, NT, [&](V (&v)[1][1 << R]) { body(v, m, lane); });
    }
}

template <typename T, int R, bool NT, typename S = T, typename Body>
__device__ __forceinline__ void jit_adj(const TileArgs &a, double *acc, Body &&body) {
    using V = cx<T>;
    const int64_t b = blockIdx.y;
    const int lane = threadIdx.x;
    const cptr<V> m = to_const((const V *)a.mats + b * a.mstride);
    adj_unit<T, R, S>((cx<S> *)a.st, (cx<S> *)a.lam, b << a.n, b << a.n, a.n, a.rbits, a.lbits, a.tbits, a.nlslots, blockIdx.x,
                   a.wps, a.partial + (b * a.wps + blockIdx.x) * (int64_t)a.ngrad, a.lslot_gslot, acc, lane, NT,
                   [&](V (&v)[2][1 << R], double *ac) { body(v, m, lane, ac); });
}

}  // namespace dq
