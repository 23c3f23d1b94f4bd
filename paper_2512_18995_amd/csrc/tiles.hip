// tiles.hip -- the register-tile passes with an op list read at run time
// (the interpreted form of a pass; a pass compiled at plan time runs the same
// operations from tile_dev.h as straight-line code).  Compiled once per
// (direction, precision): -DDQ_TILES_ADJ selects the adjoint passes (else the
// forward ones), -DDQ_TILES_F64 complex128 (else complex64), so the four
// objects build in parallel.
#include "dq_internal.h"

#include <type_traits>
#include <utility>

#ifdef DQ_TILES_F64
#define DQ_T double
#define DQ_FN(name) name##_f64
#else
#define DQ_T float
#define DQ_FN(name) name##_f32
#endif

namespace dq {
namespace {

// MultiEntry read field by field from the constant address space (scalar loads)
__device__ __forceinline__ MultiEntry ld_entry(cptr<MultiEntry> ents, int e) {
    MultiEntry E;
    E.st_off = ents[e].st_off;
    E.lam_off = ents[e].lam_off;
    E.mats_off = ents[e].mats_off;
    E.part_off = ents[e].part_off;
    E.unit_begin = ents[e].unit_begin;
    E.ops = ents[e].ops;
    E.lsg = ents[e].lsg;
    E.n = ents[e].n;
    E.nops = ents[e].nops;
    E.nls = ents[e].nls;
    E.wps = ents[e].wps;
    E.ngrad = ents[e].ngrad;
    E.nt = ents[e].nt;
    for (int k = 0; k < MAX_TILE_R; ++k) E.rbits[k] = ents[e].rbits[k];
    for (int k = 0; k < 3; ++k) E.lbits[k] = ents[e].lbits[k];
    for (int k = 0; k < MAX_TILE_R + 3; ++k) E.tbits[k] = ents[e].tbits[k];
    return E;
}

// Interpreted passes: the op list is read from memory and dispatched per op.
template <typename T, int R>
__device__ __forceinline__ void fwd_tile_ops(cx<T> *st, int64_t base, int64_t lo, const int32_t *rbits, cptr<TOp> ops,
                                             int nops, cptr<cx<T>> m, int lane, bool nt) {
    fwd_tile<T, R>(st, base, lo, rbits, nt, [&](cx<T> (&v)[1][1 << R]) {
        for (int k = 0; k < nops; ++k) apply_op<T, 1, 1 << R>(v, ld_op(ops, k), m, lane);
    });
}

template <typename T, int R>
__device__ __forceinline__ void adj_unit_ops(cx<T> *st, cx<T> *lam, int64_t sbase, int64_t lbase, int n,
                                             const int32_t *rbits, const int32_t *lbits, const int32_t *tbits,
                                             cptr<TOp> ops, int nops, int nls, cptr<cx<T>> m, int64_t w, int64_t wps,
                                             double *partial_row, const int32_t *lslot_gslot, double *acc, int lane,
                                             bool nt) {
    constexpr int NR = 1 << R;
    adj_unit<T, R>(st, lam, sbase, lbase, n, rbits, lbits, tbits, nls, w, wps, partial_row, lslot_gslot, acc, lane, nt,
                   [&](cx<T> (&v)[2][NR], double *ac) {
                       for (int k = 0; k < nops; ++k) {
                           const TOp op = ld_op(ops, k);
                           if (op.lslot >= 0) ac[op.lslot * 64 + lane] += (double)gen_local<T, NR>(v[0], v[1], op, lane);
                           apply_op<T, 2, NR>(v, op, m, lane);
                       }
                   });
}

template <typename T, int R>
__global__ __launch_bounds__(64, (tile_waves<T, R>())) void k_tile_fwd(TileArgs a) {
    using V = cx<T>;
    const int lane = threadIdx.x;
    const int tshift = a.n - 6 - R;
    const int64_t total = a.batch << tshift;
    const int64_t tmask = (int64_t(1) << tshift) - 1;
    const int64_t lo = lane_off(lane, a.lbits);
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int64_t b = tile >> tshift;
        const int64_t base = (b << a.n) + tile_base<R>(tile & tmask, a.tbits);   // wave-uniform
        fwd_tile_ops<T, R>((V *)a.st, base, lo, a.rbits, to_const(a.ops), a.nops,
                           to_const((const V *)a.mats + b * a.mstride), lane, a.nt != 0);
    }
}

template <typename T, int R>
__global__ __launch_bounds__(64, (adj_waves<T, R>())) void k_tile_adj(TileArgs a) {
    using V = cx<T>;
    extern __shared__ double acc[];   // [nlslots][64], one entry per lane
    const int64_t b = blockIdx.y;
    adj_unit_ops<T, R>((V *)a.st, (V *)a.lam, b << a.n, b << a.n, a.n, a.rbits, a.lbits, a.tbits, to_const(a.ops),
                       a.nops, a.nlslots, to_const((const V *)a.mats + b * a.mstride), blockIdx.x, a.wps,
                       a.partial + (b * a.wps + blockIdx.x) * (int64_t)a.ngrad, a.lslot_gslot, acc, threadIdx.x,
                       a.nt != 0);
}

// ---------------------------------------------------------------- uneven batches
// One launch runs the tile pass of the same depth for every circuit of a
// multi-plan: work unit u belongs to the entry e with unit_begin[e] <= u <
// unit_begin[e + 1]; pointers are base + per-entry offsets.
__device__ __forceinline__ int find_entry(cptr<MultiEntry> ents, int nent, int64_t u) {
    int lo = 0, hi = nent - 1;
    while (lo < hi) {                       // last entry with unit_begin <= u
        const int mid = (lo + hi + 1) >> 1;
        if (ents[mid].unit_begin <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T, int R>
__global__ __launch_bounds__(64, (tile_waves<T, R>())) void k_tile_fwd_multi(cx<T> *st, const char *ws,
                                                                             const MultiEntry *ents_, int nent,
                                                                             int64_t units) {
    using V = cx<T>;
    const cptr<MultiEntry> ents = to_const(ents_);
    const int lane = threadIdx.x;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int e = find_entry(ents, nent, u);
        const MultiEntry E = ld_entry(ents, e);
        const int64_t base = E.st_off + tile_base<R>(u - E.unit_begin, E.tbits);
        fwd_tile_ops<T, R>(st, base, lane_off(lane, E.lbits), E.rbits, to_const(E.ops), E.nops,
                           to_const((const V *)(ws + E.mats_off)), lane, E.nt != 0);
    }
}

template <typename T, int R>
__global__ __launch_bounds__(64, (adj_waves<T, R>())) void k_tile_adj_multi(cx<T> *st, char *ws,
                                                                            const MultiEntry *ents_, int nent) {
    using V = cx<T>;
    extern __shared__ double acc[];
    const cptr<MultiEntry> ents = to_const(ents_);
    const int64_t u = blockIdx.x;
    const int e = find_entry(ents, nent, u);
    const MultiEntry E = ld_entry(ents, e);
    const int64_t w = u - E.unit_begin;
    adj_unit_ops<T, R>(st, (V *)(ws + E.lam_off), E.st_off, 0, E.n, E.rbits, E.lbits, E.tbits, to_const(E.ops),
                       E.nops, E.nls, to_const((const V *)(ws + E.mats_off)), w, E.wps,
                       (double *)(ws + E.part_off) + w * (int64_t)E.ngrad, E.lsg, acc, threadIdx.x, E.nt != 0);
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


#ifndef DQ_TILES_ADJ
static unsigned tile_grid(int64_t tiles, int resident) {
    // one resident wave per slot; each wave walks a strided subset of the tiles
    const int64_t cap = resident > 0 ? resident : 4096;
    return (unsigned)(tiles < cap ? (tiles < 1 ? 1 : tiles) : cap);
}
#endif

}  // namespace

using T = DQ_T;

#ifndef DQ_TILES_ADJ
template <int R>
static void tile_fwd_r(const TileArgs &a, hipStream_t s) {
    const unsigned g = tile_grid(a.batch << (a.n - 6 - R), resident_waves(k_tile_fwd<T, R>, 0, R));
    hipLaunchKernelGGL((k_tile_fwd<T, R>), dim3(g), dim3(64), 0, s, a);
}

hipError_t DQ_FN(tile_fwd)(const TileArgs &a, hipStream_t s) {
    switch (a.R) {
    case 1: tile_fwd_r<1>(a, s); break;
    case 2: tile_fwd_r<2>(a, s); break;
    case 3: tile_fwd_r<3>(a, s); break;
    case 4: tile_fwd_r<4>(a, s); break;
    case 5:
        if constexpr (sizeof(T) == 4) {
            tile_fwd_r<5>(a, s);
            break;
        }
        return hipErrorInvalidValue;
    // no interpreted kernel for 64 complex64 (32 complex128) amplitudes per
    // lane: with that many and the run-time dispatch, the compiler kept the
    // tile in scratch memory; such passes are always compiled
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t DQ_FN(tile_fwd_multi)(int R, void *st, const void *ws, const MultiEntry *e, int32_t n, int64_t units,
                                 hipStream_t s) {
    const unsigned g = (unsigned)(units < 16384 ? units : 16384);
    switch (R) {
    case 3: hipLaunchKernelGGL((k_tile_fwd_multi<T, 3>), dim3(g), dim3(64), 0, s, (cx<T> *)st, (const char *)ws, e, n, units); break;
    case 4: hipLaunchKernelGGL((k_tile_fwd_multi<T, 4>), dim3(g), dim3(64), 0, s, (cx<T> *)st, (const char *)ws, e, n, units); break;
    case 5:
        if constexpr (sizeof(T) == 4) {
            hipLaunchKernelGGL((k_tile_fwd_multi<T, 5>), dim3(g), dim3(64), 0, s, (cx<T> *)st, (const char *)ws, e, n, units);
            break;
        }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#else
hipError_t DQ_FN(tile_adj)(const TileArgs &a, hipStream_t s) {
    dim3 g((unsigned)a.wps, (unsigned)a.batch);
    const size_t lds = sizeof(double) * 64 * (a.nlslots > 0 ? a.nlslots : 1);
    switch (a.R) {
    case 1: hipLaunchKernelGGL((k_tile_adj<T, 1>), g, dim3(64), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_tile_adj<T, 2>), g, dim3(64), lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_tile_adj<T, 3>), g, dim3(64), lds, s, a); break;
    case 4:
        if constexpr (sizeof(T) == 4) {
            hipLaunchKernelGGL((k_tile_adj<T, 4>), g, dim3(64), lds, s, a);
            break;
        }
        return hipErrorInvalidValue;
    // wider interpreted adjoint tiles kept their registers in scratch memory
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int DQ_FN(tile_adj_capacity)(int R) {
    const size_t lds = sizeof(double) * 64 * 32;     // the most accumulator slots a pass may use
    switch (R) {
    case 1: return resident_waves(k_tile_adj<T, 1>, lds, 8 + 1);
    case 2: return resident_waves(k_tile_adj<T, 2>, lds, 8 + 2);
    case 3: return resident_waves(k_tile_adj<T, 3>, lds, 8 + 3);
    default:
        if constexpr (sizeof(T) == 4) return resident_waves(k_tile_adj<T, 4>, lds, 8 + 4);
        return resident_waves(k_tile_adj<T, 3>, lds, 8 + 3);
    }
}

hipError_t DQ_FN(tile_adj_multi)(int R, void *st, void *ws, const MultiEntry *e, int32_t n, int64_t units, size_t lds,
                                 hipStream_t s) {
    const unsigned g = (unsigned)units;
    switch (R) {
    case 3: hipLaunchKernelGGL((k_tile_adj_multi<T, 3>), dim3(g), dim3(64), lds, s, (cx<T> *)st, (char *)ws, e, n); break;
    case 4:
        if constexpr (sizeof(T) == 4) {
            hipLaunchKernelGGL((k_tile_adj_multi<T, 4>), dim3(g), dim3(64), lds, s, (cx<T> *)st, (char *)ws, e, n);
            break;
        }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#endif

}  // namespace dq
