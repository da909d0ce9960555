// HIP kernels of the DDF executor for gfx950 (CDNA4), FP64.
//
// The paper's executor (Sec. IV-B, Listing 3) loops over partitions and, inside one, runs
// the codelets in parallel, each through the generic code of its class.  Here one
// wavefront runs a task: a range of rows of one codelet.  A codelet's record carries the
// parameters of its three access functions (Sec. III-C: f(I) = x + s[...]):
//   output row   f0: row0 + i0*row_step            or the ROWS table
//   value index  f1: op0 + i0*op_step + i1         or the OPSTART table + i1
//   input column f2: col0 + i0*sigma0 + i1*sigma1  (BLAS), col0 + i0*sigma0 + s[i1] (one
//                    shared offset table, PSC I), or a full column table (PSC II)
// so a strided function costs no index load at all and a shared table is read once per
// row group.  G lanes cooperate on one row (G = 2^lg chosen per task by the scheduler),
// 64/G rows per pass; partial sums are combined with cross-lane shuffles.
//
// The solve (Sec. IV-B: partitions in order, codelets of a partition in parallel) runs in one
// of three kernels:
//  - k_solve_df, the dataflow solve: one persistent launch with no level barriers; a row
//    waits only for the solution values it reads, each of which is its own ready flag;
//  - k_solve_thin, the single-block solve: one block runs every level, levels separated by
//    block barriers, recent solutions in an LDS ring (one right-hand side, narrow levels);
//  - k_solve_range, one launch per level (the launch boundary orders the levels).
#include <hip/hip_runtime.h>

#include <mutex>

#include "ddf_internal.hpp"
#include "kernels.hpp"

namespace ddf {
namespace {

constexpr int WAVE = 64;
constexpr int WPB = 4; // waves per block (256 threads)

__device__ __forceinline__ double cload(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cstore(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned cload_u(const unsigned *p) {
    return __hip_atomic_load(const_cast<unsigned *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// column-table mode of a codelet
enum : int { XM_STRIDED = 0, XM_SHARED = 1, XM_SHARED_RUNS = 2, XM_FULL = 3, XM_FULL_RUNS = 4 };

__device__ __forceinline__ int xmode(int flags) {
    if (flags & FS2) return XM_STRIDED;
    if (flags & FSEP) return (flags & FRUNS) ? XM_SHARED_RUNS : XM_SHARED;
    return (flags & FRUNS) ? XM_FULL_RUNS : XM_FULL;
}

struct RowInfo {
    int row, opst, nops;
};

__device__ __forceinline__ RowInfo row_info(const DCod &c, const int32_t *__restrict__ aux, int i0) {
    RowInfo r;
    r.row = (c.flags & FS0) ? c.row0 + i0 * c.row_step : aux[c.rows_off + i0];
    r.opst = (c.flags & DOPS) ? aux[c.ops_off + i0] : c.op0 + i0 * c.op_step;
    r.nops = (c.flags & FRECT) ? c.nn : aux[c.cnt_off + i0];
    return r;
}

// Calls f(value index, column) for the ops i1 = g, g+G, ... of row i0, in that order.  U4:
// column tables are read four ops at a time before the calls, so that four ops' loads are in
// flight (the solve tasks; for SpMV tasks the extra registers cost more than they hide).
template <int MODE, bool U4 = false, class F>
__device__ __forceinline__ void walk(const DCod &c, const int32_t *__restrict__ aux, int i0,
                                     const RowInfo &ri, int g, int G, F &&f) {
    if constexpr (MODE == XM_STRIDED) {
        const int base = c.col0 + i0 * c.sigma0;
        for (int i1 = g; i1 < ri.nops; i1 += G) f(ri.opst + i1, base + i1 * c.sigma1);
    } else if constexpr (MODE == XM_SHARED || MODE == XM_FULL) {
        int base = 0;
        const int32_t *__restrict__ s;
        if constexpr (MODE == XM_SHARED) {
            base = c.col0 + i0 * c.sigma0;
            s = aux + c.xt_off;
        } else {
            int off;
            if (c.flags & FRECT)
                off = i0 * c.nn;
            else if (c.flags & DCONTIG)
                off = ri.opst - c.op0;
            else
                off = aux[c.xp_off + i0];
            s = aux + c.xt_off + off;
        }
        int i1 = g;
        if constexpr (U4)
            for (; i1 + 3 * G < ri.nops; i1 += 4 * G) {
                const int c0 = s[i1], c1 = s[i1 + G], c2 = s[i1 + 2 * G], c3 = s[i1 + 3 * G];
                f(ri.opst + i1, base + c0);
                f(ri.opst + i1 + G, base + c1);
                f(ri.opst + i1 + 2 * G, base + c2);
                f(ri.opst + i1 + 3 * G, base + c3);
            }
        for (; i1 < ri.nops; i1 += G) f(ri.opst + i1, base + s[i1]);
    } else {
        const int32_t *__restrict__ rt;
        int base;
        if constexpr (MODE == XM_SHARED_RUNS) {
            rt = aux + c.xt_off;
            base = c.col0 + i0 * c.sigma0;
        } else {
            rt = aux + c.xt_off + 2 * aux[c.xp_off + i0];
            base = 0;
        }
        int j = -1, cum = 0, ln = 0, st = 0;
        for (int i1 = g; i1 < ri.nops; i1 += G) {
            while (i1 >= cum + ln) {
                cum += ln;
                ++j;
                st = rt[2 * j];
                ln = rt[2 * j + 1];
            }
            f(ri.opst + i1, base + st + (i1 - cum));
        }
    }
}

template <bool U4 = false, class F>
__device__ __forceinline__ void walk_any(int mode, const DCod &c, const int32_t *__restrict__ aux, int i0,
                                         const RowInfo &ri, int g, int G, F &&f) {
    switch (mode) {
    case XM_STRIDED: walk<XM_STRIDED, U4>(c, aux, i0, ri, g, G, f); break;
    case XM_SHARED: walk<XM_SHARED, U4>(c, aux, i0, ri, g, G, f); break;
    case XM_SHARED_RUNS: walk<XM_SHARED_RUNS, U4>(c, aux, i0, ri, g, G, f); break;
    case XM_FULL: walk<XM_FULL, U4>(c, aux, i0, ri, g, G, f); break;
    default: walk<XM_FULL_RUNS, U4>(c, aux, i0, ri, g, G, f); break;
    }
}

template <int KT>
__device__ __forceinline__ void group_sum(double (&acc)[KT], int G) {
    for (int s = 1; s < G; s <<= 1)
#pragma unroll
        for (int r = 0; r < KT; r++) acc[r] += __shfl_xor(acc[r], s, WAVE);
}

__device__ __forceinline__ int xcd_block(int b, int nb, int remap) {
    if (!remap) return b;
    // blocks are dispatched round-robin over the 8 XCDs; give XCD x a contiguous range
    const int q = nb >> 3, rr = nb & 7, x = b & 7;
    return x * q + min(x, rr) + (b >> 3);
}

__device__ __forceinline__ DCod load_cod(const DCod *p) { return *p; }

// Task list entries and codelet copies through the constant address space: scalar loads where
// the index is wave-uniform (16-byte vectors, since structs cannot be copied out of that space).
typedef int dfv4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) dfv4 *const_v4_ptr;
typedef const __attribute__((address_space(4))) int *const_i32k_ptr;

__device__ __forceinline__ Task k_task(const Task *tasks, int i) {
    const dfv4 v = ((const_v4_ptr)tasks)[i];
    return Task{v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ DCod k_cod(const DCod *cods, int i) {
    const const_v4_ptr p = (const_v4_ptr)cods + 4 * (int64_t)i;
    const dfv4 a = p[0], b = p[1], c = p[2], d = p[3];
    return DCod{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
}


// ------------------------------------------------------------------------------------------
// SpMV executor.  Three task shapes, chosen per task by the scheduler:
//  - stream (one right-hand side, rectangular codelet with contiguous values): the task's
//    values (and a full column table) are one contiguous range; lane l takes elements
//    l + 64 j, keeps SJ independent loads in flight, and row sums go through LDS;
//  - lanes-per-row (one right-hand side, any codelet): G lanes share a row, shuffles
//    combine their partial sums;
//  - rhs-lanes (several right-hand sides): KR lanes per row, lane r owns right-hand side r,
//    so each x row is read as one contiguous 8*k-byte segment and no reduction is needed.
// VPERM reads values through perm (the transposed plan of the adjoint pass).
// ------------------------------------------------------------------------------------------
constexpr int SJ = 8; // elements per lane of a stream task (64 * SJ per task)

template <bool VPERM>
__device__ __forceinline__ double val_at(const SpmvArgs &a, int e) {
    return VPERM ? a.vals[a.perm[e]] : a.vals[e];
}

__device__ __forceinline__ int row_of(const DCod &c, const int32_t *__restrict__ aux, int i0) {
    return (c.flags & FS0) ? c.row0 + i0 * c.row_step : aux[c.rows_off + i0];
}

template <int MODE, bool VPERM>
__device__ __forceinline__ void spmv_stream_body(const SpmvArgs &a, const DCod &c, int a0, int nrow, int lane,
                                                 double *__restrict__ lds) {
    const int nn = c.nn, E = nrow * nn;
    const int ebase = c.op0 + a0 * nn;
    // q = e / nn as (e * ceil(2^32 / nn)) >> 32: exact for e, nn < 2^16
    const uint64_t magic = 0xFFFFFFFFull / (uint64_t)nn + 1ull;
    // every load is unconditional (indices clamped into the task) so that a lane issues all
    // of its value, column and then x loads back to back
    int col[SJ];
    double v[SJ];
#pragma unroll
    for (int j = 0; j < SJ; j++) {
        const int e = min(lane + WAVE * j, E - 1);
        const int q = (int)(((uint64_t)e * magic) >> 32);
        const int i1 = e - q * nn;
        const int i0 = a0 + q;
        if constexpr (MODE == XM_STRIDED)
            col[j] = c.col0 + i0 * c.sigma0 + i1 * c.sigma1;
        else if constexpr (MODE == XM_SHARED)
            col[j] = c.col0 + i0 * c.sigma0 + a.aux[c.xt_off + i1];
        else
            col[j] = a.aux[c.xt_off + a0 * nn + e];
        // a wave reads whole lines of values exactly once: non-temporal loads leave the L2 to x
        v[j] = VPERM ? val_at<VPERM>(a, ebase + e) : __builtin_nontemporal_load(a.vals + ebase + e);
    }
    double xv[SJ];
#pragma unroll
    for (int j = 0; j < SJ; j++) xv[j] = a.x[col[j]];
#pragma unroll
    for (int j = 0; j < SJ; j++) {
        const int e = lane + WAVE * j;
        if (e < E) lds[e] = v[j] * xv[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < nrow) {
        double s = 0.0;
        for (int i1 = 0; i1 < nn; i1++) s += lds[lane * nn + i1];
        a.y[row_of(c, a.aux, a0 + lane)] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool VPERM>
__device__ __forceinline__ void spmv_stream_task(const SpmvArgs &a, const Task &tk, int lane, double *__restrict__ lds) {
    const DCod c = k_cod(a.cods, tk.cod);
    const int mode = xmode(c.flags);
    if (mode == XM_STRIDED)
        spmv_stream_body<XM_STRIDED, VPERM>(a, c, tk.i0b, tk.i0e - tk.i0b, lane, lds);
    else if (mode == XM_SHARED)
        spmv_stream_body<XM_SHARED, VPERM>(a, c, tk.i0b, tk.i0e - tk.i0b, lane, lds);
    else
        spmv_stream_body<XM_FULL, VPERM>(a, c, tk.i0b, tk.i0e - tk.i0b, lane, lds);
}

template <bool VPERM>
__device__ __forceinline__ void spmv_group_task(const SpmvArgs &a, const Task &tk, int lane) {
    const DCod c = k_cod(a.cods, tk.cod);
    const int lg = tk.meta & 7, G = 1 << lg, R = WAVE >> lg;
    const int slot = lane >> lg, g = lane & (G - 1);
    const int mode = xmode(c.flags);
    for (int base = tk.i0b; base < tk.i0e; base += R) {
        const int i0 = base + slot;
        const bool active = i0 < tk.i0e;
        RowInfo ri{0, 0, 0};
        if (active) ri = row_info(c, a.aux, i0);
        double acc[1] = {0.0};
        if (active) walk_any(mode, c, a.aux, i0, ri, g, G, [&](int e, int col) { acc[0] += val_at<VPERM>(a, e) * a.x[col]; });
        group_sum<1>(acc, G);
        if (active && g == 0) a.y[ri.row] = acc[0];
    }
}

// Rows [r0, r1) of the CSR pattern, one right-hand side: elements streamed like a stream task
// (products into LDS, then one lane per row sums), or one long row in chunks with a wave sum.
template <bool VPERM>
__device__ void spmv_csr_task(const SpmvArgs &a, const Task &tk, int lane, double *__restrict__ lds) {
    const int r0 = tk.i0b, r1 = tk.i0e;
    const int e0 = a.rp[r0], e1 = a.rp[r1];
    if (tk.meta & TASK_LONG) {
        double acc = 0.0;
        for (int base = e0; base < e1; base += WAVE * SJ) {
            int col[SJ];
            double v[SJ];
#pragma unroll
            for (int j = 0; j < SJ; j++) {
                const int e = min(base + lane + WAVE * j, e1 - 1);
                col[j] = a.ci[e];
                v[j] = VPERM ? a.vals[a.perm[e]] : __builtin_nontemporal_load(a.vals + e);
            }
            double xv[SJ];
#pragma unroll
            for (int j = 0; j < SJ; j++) xv[j] = a.x[col[j]];
#pragma unroll
            for (int j = 0; j < SJ; j++)
                if (base + lane + WAVE * j < e1) acc += v[j] * xv[j];
        }
        double t[1] = {acc};
        group_sum<1>(t, WAVE);
        if (lane == 0) a.y[r0] = t[0];
        return;
    }
    const int E = e1 - e0, nrow = r1 - r0;
    if (E == 0) {
        if (lane < nrow) a.y[r0 + lane] = 0.0;
        return;
    }
    int col[SJ];
    double v[SJ];
#pragma unroll
    for (int j = 0; j < SJ; j++) {
        const int e = e0 + min(lane + WAVE * j, E - 1);
        col[j] = a.ci[e];
        v[j] = VPERM ? a.vals[a.perm[e]] : __builtin_nontemporal_load(a.vals + e);
    }
    double xv[SJ];
#pragma unroll
    for (int j = 0; j < SJ; j++) xv[j] = a.x[col[j]];
#pragma unroll
    for (int j = 0; j < SJ; j++)
        if (lane + WAVE * j < E) lds[lane + WAVE * j] = v[j] * xv[j];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < nrow) {
        const int b0 = a.rp[r0 + lane] - e0, b1 = a.rp[r0 + lane + 1] - e0;
        double sum = 0.0;
        for (int q = b0; q < b1; q++) sum += lds[q];
        a.y[r0 + lane] = sum;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Scattered short rows from the CSR pattern, one lane per row of list[i0b, i0e): packs the
// rows of small codelets that no run of consecutive rows covers, 64 to a wave.
template <bool VPERM> __device__ void spmv_rows_task(const SpmvArgs &a, const Task &tk, int lane) {
    const int i = tk.i0b + lane;
    if (i >= tk.i0e) return;
    const int row = a.rows[i];
    const int e0 = a.rp[row], e1 = a.rp[row + 1];
    double acc = 0.0;
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
        int c[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            c[u] = a.ci[e + u];
            v[u] = val_at<VPERM>(a, e + u);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) acc = fma(v[u], a.x[c[u]], acc);
    }
    for (; e < e1; e++) acc = fma(val_at<VPERM>(a, e), a.x[a.ci[e]], acc);
    a.y[row] = acc;
}

// one right-hand side: stream and lanes-per-row tasks
template <bool VPERM>
__global__ __launch_bounds__(WAVE *WPB) void k_spmv1(SpmvArgs a) {
    __shared__ double lds_all[WPB][WAVE * SJ];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int t = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x, a.remap) * WPB + wave);
    if (t >= a.ntasks) return;
    const Task tk = k_task(a.tasks, t);
    if (tk.meta & TASK_CSR)
        spmv_csr_task<VPERM>(a, tk, lane, lds_all[wave]);
    else if (tk.meta & TASK_ROWS)
        spmv_rows_task<VPERM>(a, tk, lane);
    else if (tk.meta & TASK_STREAM)
        spmv_stream_task<VPERM>(a, tk, lane, lds_all[wave]);
    else
        spmv_group_task<VPERM>(a, tk, lane);
}

// several right-hand sides: KR lanes per row, lane r owns right-hand sides r, r + KR, ...
constexpr int RU = 4;  // ops per unrolled chunk of a rectangular row (one RHS per lane)
// the same with RV right-hand sides per lane (16-byte loads); a chunk past the row's end
// repeats its last operand, so 7 wastes no load on 7-point rows and one on 27-point rows
// (27-point Laplacian on 170^3, 8 right-hand sides: 0.78 ms with 8, 0.74 with 6, 0.72 with 7)
constexpr int RUV = 7;

template <int KR, int MODE, bool VPERM>
__device__ __forceinline__ void spmvN_rect(const SpmvArgs &a, const DCod &c, const Task &tk, int lane) {
    constexpr int P = WAVE / KR;
    const int slot = lane / KR, r = lane % KR;
    const int k = a.k, nn = c.nn;
    for (int base = tk.i0b; base < tk.i0e; base += P) {
        const int i0 = min(base + slot, tk.i0e - 1);
        const bool active = base + slot < tk.i0e;
        const int row = row_of(c, a.aux, i0);
        const int opst = c.op0 + i0 * c.op_step;
        const int cbase = (MODE == XM_FULL) ? c.xt_off + i0 * nn : c.col0 + i0 * c.sigma0;
        for (int r0 = 0; r0 < k; r0 += KR) {
            const int rr = min(r0 + r, k - 1);
            double acc = 0.0;
            for (int i1 = 0; i1 < nn; i1 += RU) {
                int col[RU];
                double v[RU], xv[RU];
#pragma unroll
                for (int u = 0; u < RU; u++) {
                    const int j = min(i1 + u, nn - 1);
                    if constexpr (MODE == XM_STRIDED)
                        col[u] = cbase + j * c.sigma1;
                    else if constexpr (MODE == XM_SHARED)
                        col[u] = cbase + ((const_i32k_ptr)a.aux)[c.xt_off + j];
                    else
                        col[u] = a.aux[cbase + j];
                    v[u] = val_at<VPERM>(a, opst + j);
                }
#pragma unroll
                for (int u = 0; u < RU; u++) xv[u] = a.x[(int64_t)col[u] * k + rr];
#pragma unroll
                for (int u = 0; u < RU; u++)
                    if (i1 + u < nn) acc += v[u] * xv[u];
            }
            if (active && r0 + r < k) a.y[(int64_t)row * k + r0 + r] = acc;
        }
    }
}

// Rectangular codelet, RV consecutive right-hand sides per lane (vector loads of x and y),
// KR lanes per row.  STG: the codelet's ops are row-major and contiguous (op_step == nn) and
// P rows of them fit the wave's LDS slice sv: the wave first copies the values of its P rows
// there with coalesced loads (a row's nn values are nn * 8 bytes apart from the next row's, so
// direct loads would touch a cache line per row), then reads them from LDS.
constexpr int SV_CAP = 1024; // doubles of LDS per wave for staged values

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KR, int RV, int MODE, bool VPERM, bool STG>
__device__ __forceinline__ void spmvN_rect_v(const SpmvArgs &a, const DCod &c, const Task &tk, int lane, double *sv) {
    static_assert(RV == 2 || RV == 4, "vector width");
    constexpr int P = WAVE / KR;
    constexpr int SU = SV_CAP / WAVE;
    const int slot = lane / KR, r = (lane % KR) * RV;
    const int k = a.k, nn = c.nn;
    for (int base = tk.i0b; base < tk.i0e; base += P) {
        const int i0 = min(base + slot, tk.i0e - 1);
        const bool active = base + slot < tk.i0e;
        const int row = row_of(c, a.aux, i0);
        const int opst = c.op0 + i0 * c.op_step;
        const int cbase = (MODE == XM_FULL) ? c.xt_off + i0 * nn : c.col0 + i0 * c.sigma0;
        if constexpr (STG) {
            const int e0 = c.op0 + base * nn, ne = min(P, tk.i0e - base) * nn;
            double t[SU];
#pragma unroll
            for (int u = 0; u < SU; u++) {
                const int q = lane + u * WAVE;
                t[u] = q < ne ? val_at<VPERM>(a, e0 + q) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < SU; u++) {
                const int q = lane + u * WAVE;
                if (q < ne) sv[q] = t[u];
            }
            wave_sync();
        }
        double acc[RV];
#pragma unroll
        for (int q = 0; q < RV; q++) acc[q] = 0.0;
        for (int i1 = 0; i1 < nn; i1 += RUV) {
            int col[RUV];
            double v[RUV];
            double2 xv[RUV][RV / 2];
#pragma unroll
            for (int u = 0; u < RUV; u++) {
                const int j = min(i1 + u, nn - 1);
                if constexpr (MODE == XM_STRIDED)
                    col[u] = cbase + j * c.sigma1;
                else if constexpr (MODE == XM_SHARED)
                    col[u] = cbase + ((const_i32k_ptr)a.aux)[c.xt_off + j];
                else
                    col[u] = a.aux[cbase + j];
                if constexpr (STG)
                    v[u] = sv[(i0 - base) * nn + j];
                else
                    v[u] = val_at<VPERM>(a, opst + j);
            }
#pragma unroll
            for (int u = 0; u < RUV; u++) {
                const double2 *xp = reinterpret_cast<const double2 *>(a.x + (int64_t)col[u] * k + r);
#pragma unroll
                for (int h = 0; h < RV / 2; h++) xv[u][h] = xp[h];
            }
#pragma unroll
            for (int u = 0; u < RUV; u++)
                if (i1 + u < nn) {
#pragma unroll
                    for (int h = 0; h < RV / 2; h++) {
                        acc[2 * h] += v[u] * xv[u][h].x;
                        acc[2 * h + 1] += v[u] * xv[u][h].y;
                    }
                }
        }
        if (active) {
            double2 *yp = reinterpret_cast<double2 *>(a.y + (int64_t)row * k + r);
#pragma unroll
            for (int h = 0; h < RV / 2; h++) yp[h] = make_double2(acc[2 * h], acc[2 * h + 1]);
        }
        if constexpr (STG) wave_sync();
    }
}

template <int KR, bool VPERM>
__device__ __forceinline__ void spmvN_walk(const SpmvArgs &a, const DCod &c, const Task &tk, int lane) {
    constexpr int P = WAVE / KR;
    const int slot = lane / KR, r = lane % KR;
    const int k = a.k;
    const int mode = xmode(c.flags);
    for (int base = tk.i0b; base < tk.i0e; base += P) {
        const int i0 = base + slot;
        if (i0 >= tk.i0e) break;
        const RowInfo ri = row_info(c, a.aux, i0);
        for (int r0 = 0; r0 < k; r0 += KR) {
            const int rr = r0 + r;
            if (rr >= k) break;
            double acc = 0.0;
            walk_any(mode, c, a.aux, i0, ri, 0, 1,
                     [&](int e, int col) { acc += val_at<VPERM>(a, e) * a.x[(int64_t)col * k + rr]; });
            a.y[(int64_t)ri.row * k + rr] = acc;
        }
    }
}

// KR lanes per row; RV > 1: rectangular codelets take RV right-hand sides per lane (k is
// KR * RV), others one per lane over KW lanes per row
template <int KR, int RV, int KW, bool VPERM>
__global__ __launch_bounds__(WAVE *WPB, 4) void k_spmvN(SpmvArgs a) {
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    // a task per wave: its index is wave-uniform, the task and its codelet record come with
    // scalar loads, and so do the codelet's shared column offsets
    const int t = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x, a.remap) * WPB + wave);
    if (t >= a.ntasks) return;
    const Task tk = k_task(a.tasks, t);
    const DCod c = k_cod(a.cods, tk.cod);
    const int mode = xmode(c.flags);
    const bool rect = (c.flags & FRECT) && !(c.flags & DOPS) && c.nn > 0;
    if constexpr (RV > 1) {
        __shared__ double sv_all[WPB][SV_CAP];
        double *sv = sv_all[wave];
        const bool stg = c.op_step == c.nn && (WAVE / KR) * c.nn <= SV_CAP;
        if (rect && stg && mode == XM_SHARED)
            spmvN_rect_v<KR, RV, XM_SHARED, VPERM, true>(a, c, tk, lane, sv);
        else if (rect && stg && mode == XM_STRIDED)
            spmvN_rect_v<KR, RV, XM_STRIDED, VPERM, true>(a, c, tk, lane, sv);
        else if (rect && stg && mode == XM_FULL)
            spmvN_rect_v<KR, RV, XM_FULL, VPERM, true>(a, c, tk, lane, sv);
        else if (rect && mode == XM_STRIDED)
            spmvN_rect_v<KR, RV, XM_STRIDED, VPERM, false>(a, c, tk, lane, sv);
        else if (rect && mode == XM_SHARED)
            spmvN_rect_v<KR, RV, XM_SHARED, VPERM, false>(a, c, tk, lane, sv);
        else if (rect && mode == XM_FULL)
            spmvN_rect_v<KR, RV, XM_FULL, VPERM, false>(a, c, tk, lane, sv);
        else
            spmvN_walk<KW, VPERM>(a, c, tk, lane);
    } else {
        if (rect && mode == XM_STRIDED)
            spmvN_rect<KR, XM_STRIDED, VPERM>(a, c, tk, lane);
        else if (rect && mode == XM_SHARED)
            spmvN_rect<KR, XM_SHARED, VPERM>(a, c, tk, lane);
        else if (rect && mode == XM_FULL)
            spmvN_rect<KR, XM_FULL, VPERM>(a, c, tk, lane);
        else
            spmvN_walk<KR, VPERM>(a, c, tk, lane);
    }
}

// ------------------------------------------------------------------------------------------
// Solve task body shared by the per-level kernel (k_solve_range): every row of one task, all
// passes, all right-hand-side tiles (forward L x = b, or the adjoint U lam = g with U = L^T).
// ------------------------------------------------------------------------------------------
// A single-matrix call's bases are zero: no load on the task's dependent chain for them.
__device__ __forceinline__ MatInfo mat_info(const SolveArgs &a, const DCod &c) {
    if (a.k_override > 0) return MatInfo{0, 0, 0, a.k_override, 0};
    return a.mats[c.mat];
}

template <bool COH>
__device__ __forceinline__ double xload(const double *p) {
    if constexpr (COH) return cload(p);
    else return *p;
}
template <bool COH>
__device__ __forceinline__ void xstore(double *p, double v) {
    if constexpr (COH) cstore(p, v);
    else *p = v;
}

// every row of one task, all passes, all right-hand-side tiles
// SINGLE (the per-level kernel of a single-matrix call): ops' column reads run four ahead, and
// the adjoint's values come in U's order (gathered before the solve), not through perm.
template <int KT, bool ADJ, bool COH, bool SINGLE = false>
__device__ void solve_task(const SolveArgs &a, int t, int lane) {
    const Task tk = a.tasks[t];
    const DCod c = a.tcods ? a.tcods[t] : load_cod(a.cods + tk.cod);
    const MatInfo mi = mat_info(a, c);
    const int lg = tk.meta & 7, G = 1 << lg, R = WAVE >> lg;
    const int slot = lane >> lg, g = lane & (G - 1);
    const int k = a.k_override > 0 ? a.k_override : mi.k;
    const double *__restrict__ vals = a.vals + mi.val_base;
    const int mode = xmode(c.flags);
    constexpr bool VP = ADJ && !SINGLE; // values through perm
    const int32_t *__restrict__ perm = VP ? a.perm + mi.val_base : nullptr;
    const double *__restrict__ b = a.b + mi.vec_base;
    double *x = a.x + mi.vec_base;
    for (int base = tk.i0b; base < tk.i0e; base += R) {
        const int i0 = base + slot;
        const bool active = i0 < tk.i0e;
        RowInfo ri{0, 0, 0};
        double diag = 1.0;
        if (active) {
            ri = row_info(c, a.aux, i0);
            const int dpos = ADJ ? ri.opst - 1 : ri.opst + ri.nops;
            diag = VP ? vals[perm[dpos]] : vals[dpos];
        }
        const int64_t rb = (int64_t)ri.row * k;
        for (int r0 = 0; r0 < k; r0 += KT) {
            double acc[KT];
#pragma unroll
            for (int r = 0; r < KT; r++) acc[r] = 0.0;
            if (active)
                walk_any<SINGLE>(mode, c, a.aux, i0, ri, g, G, [&](int e, int col) {
                    const double v = VP ? vals[perm[e]] : vals[e];
                    const double *xr = x + (int64_t)col * k + r0;
#pragma unroll
                    for (int r = 0; r < KT; r++)
                        if (r0 + r < k) acc[r] += v * xload<COH>(xr + r);
                });
            group_sum<KT>(acc, G);
            if (active) {
#pragma unroll
                for (int r = 0; r < KT; r++)
                    if ((r & (G - 1)) == g && r0 + r < k) xstore<COH>(x + rb + r0 + r, (b[rb + r0 + r] - acc[r]) / diag);
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Dataflow solve: the whole solve (or transposed solve) in one persistent launch, with no
// level barriers.  Each solution value is its own ready flag: before the launch the output
// is filled with DF_SENT, a signalling NaN that no arithmetic result has (results are
// quiet NaNs), and a task loads the solution values its rows need first through the caches
// (wload), then re-reads those that still hold the sentinel with device-coherent loads
// (agent-scope relaxed atomics, which bypass the per-XCD caches), with backoff; it stores its
// own results with device-coherent stores.  Every location is written once, after the fill,
// and the launch starts with caches that hold nothing older than the fill, so a cached copy
// is the sentinel or the final value; an 8-byte store is seen whole, so a value that is not
// the sentinel is final: no counters, fences or flags are needed.
//
// A task is up to DF_RG rows of one codelet; tasks are in level order, a topological order of
// the dependences.  KR lanes per row each own right-hand sides r, r + KR, ...; a pass of a
// wave covers 64 / KR rows, that is 64 / (KR DF_RG) consecutive tasks.  The blocks first
// check in: when all of them are resident at once, wave w runs passes w, w + V, w + 2V, ... of
// the V waves (no atomics at all); when some are not (another kernel holds part of the
// device), the first block to give up waiting switches every wave to passes taken in order
// from an atomic ticket.  Either way the earliest unfinished task is held by a running wave
// whose dependences are all complete, so the solve always progresses.  A wait longer than
// the plan's spin limit raises the plan's error flag and stops waiting (the results are then
// reported invalid by ddf_plan_sync_status); once the flag is up every wave stops waiting.
// ------------------------------------------------------------------------------------------
constexpr unsigned long long DF_SENT_BITS = 0x7FF4DDF0DDF0DDF0ull; // signalling NaN
constexpr int DF_ARRIVE_POLLS = 400;                                 // check-in wait (~0.3 ms)

// First read of a solution value: a relaxed load at workgroup scope, which the per-CU and
// per-XCD caches may serve.  A location holds only the sentinel (written before the launch)
// or its final value (written once), so a cached copy is either final or the sentinel; the
// sentinel is then re-read from the device-coherent level (cload) until it is final.
__device__ __forceinline__ double wload(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ bool df_missing(double v) {
    return (unsigned long long)__double_as_longlong(v) == DF_SENT_BITS;
}

// Columns of one row's ops, for every column-table mode, in ascending op order, or descending
// (DESC).  In the run mode the op index must move by one from call to call (up, or down from
// the last op); the other modes take any order.
template <bool DESC> struct ColIter {
    int mode, base, j, cum, ln, st;
    const int32_t *__restrict__ s;
    __device__ __forceinline__ void init(const DCod &c, const int32_t *__restrict__ aux, int i0, const RowInfo &ri) {
        mode = xmode(c.flags);
        j = -1;
        cum = ln = st = 0;
        base = 0;
        s = aux;
        if (mode == XM_STRIDED || mode == XM_SHARED || mode == XM_SHARED_RUNS) base = c.col0 + i0 * c.sigma0;
        if (mode == XM_SHARED || mode == XM_SHARED_RUNS) s = aux + c.xt_off;
        else if (mode == XM_FULL) {
            const int off = (c.flags & FRECT) ? i0 * c.nn : (c.flags & DCONTIG) ? ri.opst - c.op0 : aux[c.xp_off + i0];
            s = aux + c.xt_off + off;
        } else if (mode == XM_FULL_RUNS) {
            s = aux + c.xt_off + 2 * aux[c.xp_off + i0];
            if (DESC) { // start past the row's last run (the run index table has one more entry)
                j = aux[c.xp_off + i0 + 1] - aux[c.xp_off + i0];
                cum = ri.nops;
            }
        }
    }
    __device__ __forceinline__ int col(const DCod &c, int i1) {
        if (mode == XM_STRIDED) return base + i1 * c.sigma1;
        if (mode == XM_SHARED || mode == XM_FULL) return base + s[i1];
        if (DESC) {
            while (i1 < cum) {
                --j;
                st = s[2 * j];
                ln = s[2 * j + 1];
                cum -= ln;
            }
        } else {
            while (i1 >= cum + ln) {
                cum += ln;
                ++j;
                st = s[2 * j];
                ln = s[2 * j + 1];
            }
        }
        return base + st + (i1 - cum);
    }
};

// Re-reads the values that still hold the sentinel, with backoff; returns false once the
// wait has tripped the watchdog (the spin limit, or the error flag raised by another wave).
template <int U>
__device__ __forceinline__ bool df_backoff(const SolveArgs &a, int64_t &spins, int &back, unsigned *err) {
    for (int z = 0; z < back; z++) __builtin_amdgcn_s_sleep(1);
    if (back < a.backoff_max) back <<= 1;
    spins += back;
    bool trip = spins > a.spin_limit;
    if ((spins & 1023) < back) trip = trip || cload_u(err) != 0u;
    if (__ballot(trip)) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
    }
    return true;
}

// Re-reads a lane's missing solution values.  ALL: every one of them.  Otherwise only the last
// missing one, which is normally the latest dependence since a lane's ops run in dependence
// order, and once it has arrived the others still missing at once: a wait then costs one load
// per lane and poll rather than one per missing value.  With one or two right-hand sides a pass
// holds 32 or 64 rows, one or two lanes each, whose polls hit different lines: polling only
// the last keeps the many waiting waves from crowding the memory system (27-point Laplacian
// on 170^3, one right-hand side: 19.3 ms -> 4.8 ms).  With more right-hand sides the lanes of
// a row poll one line together and the extra round trip after the last arrival costs more
// than the polls (eight right-hand sides: 3.1 ms -> 4.3 ms).
template <int U, bool ALL>
__device__ __forceinline__ void df_poll(double (&xv)[U], const int (&col)[U], const double *x, int k, int rr) {
    if constexpr (ALL) {
#pragma unroll
        for (int u = 0; u < U; u++)
            if (df_missing(xv[u])) xv[u] = cload(x + (int64_t)col[u] * k + rr);
        return;
    }
    int last = -1;
#pragma unroll
    for (int u = 0; u < U; u++)
        if (df_missing(xv[u])) last = u;
    bool got = false;
#pragma unroll
    for (int u = 0; u < U; u++)
        if (u == last) {
            xv[u] = cload(x + (int64_t)col[u] * k + rr);
            got = !df_missing(xv[u]);
        }
    if (got) {
#pragma unroll
        for (int u = 0; u < U; u++)
            if (u != last && df_missing(xv[u])) xv[u] = cload(x + (int64_t)col[u] * k + rr);
    }
}

// A row's result from its values and the solution values it reads: stored for the readers.
template <int U>
__device__ __forceinline__ void df_finish(const double (&v)[U], const double (&xv)[U], double acc, double bo,
                                          double diag, double *dst) {
#pragma unroll
    for (int u = 0; u < U; u++) acc = fma(v[u], xv[u], acc);
    double res = (bo - acc) / diag;
    if (df_missing(res)) res = __longlong_as_double(0x7FF8000000000000ll); // never: results are quiet
    cstore(dst, res);
}

// A wide-row task (DF_LONG) with the whole wave: its R rows (R up to 8) take 64 / R' lanes each
// (R' = R rounded up to a power of two); of a row's lanes, KL = min(k rounded up to a power of
// two, lanes) own right-hand sides r, r + KL, ..., and the GR = lanes / KL groups of them split
// the row's ops (in each chunk of GR x DF_U ops, group j takes ops j, j + GR, ...).  The
// groups' sums are combined with cross-lane shuffles and the first group stores the row.  The
// task's rows keep their columns one after the other in lcols (ascending op order; the
// transposed solve walks the ops from the last, as the other rows do).
template <bool ADJ, bool VPERM>
__device__ __forceinline__ void df_long(const SolveArgs &a, const Task &tk, const DCod &c, int lane) {
    const int nrow = (tk.meta >> DF_LONG_ROWS_SHIFT) & 15;
    const int lgr = nrow <= 1 ? 0 : nrow <= 2 ? 1 : nrow <= 4 ? 2 : 3;
    const int lanes = WAVE >> lgr;
    const MatInfo mi = mat_info(a, c);
    const int k = mi.k;
    int kl = 1;
    while (kl < k && kl < lanes) kl <<= 1;
    const int gr = lanes / kl;
    const int ri_idx = lane / lanes, sub = lane % lanes;
    const int r = sub % kl, gq = sub / kl;
    const bool row_on = ri_idx < nrow;
    const double *__restrict__ vals = a.vals + mi.val_base;
    const int32_t *__restrict__ perm = VPERM ? a.perm + mi.val_base : nullptr;
    const double *__restrict__ b = a.b + mi.vec_base;
    double *x = a.x + mi.vec_base;
    RowInfo ri{0, 0, 0};
    int coff = tk.i0e; // this row's columns: after those of the task's earlier rows
    double diag = 1.0;
    if (row_on) {
        for (int j = 0; j < ri_idx; j++) coff += row_info(c, a.aux, tk.i0b + j).nops;
        ri = row_info(c, a.aux, tk.i0b + ri_idx);
        const int dpos = ADJ ? ri.opst - 1 : ri.opst + ri.nops;
        diag = VPERM ? vals[perm[dpos]] : vals[dpos];
    }
    const int32_t *__restrict__ cols = a.lcols + coff;
    unsigned *err = a.err ? a.err : a.ctr + CTR_STRIDE;
    bool live = true; // false once the watchdog has tripped
    for (int r0 = 0; r0 < k; r0 += kl) {
        const int rr = r0 + r;
        const bool mine = row_on && rr < k;
        const int nops = mine ? ri.nops : 0;
        double acc = 0.0;
        for (int i1 = 0; __ballot(i1 < nops); i1 += gr * DF_U) {
            double v[DF_U], xv[DF_U];
            int col[DF_U];
#pragma unroll
            for (int u = 0; u < DF_U; u++) {
                const int q = i1 + u * gr + gq;
                const bool ok = q < nops;
                const int op = ADJ ? nops - 1 - q : q;
                col[u] = ok ? cols[op] : 0;
                const int e = ri.opst + op;
                v[u] = ok ? (VPERM ? vals[perm[e]] : vals[e]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < DF_U; u++)
                xv[u] = i1 + u * gr + gq < nops ? wload(x + (int64_t)col[u] * k + rr) : 0.0;
            int64_t spins = 0;
            int back = 1;
            for (;;) {
                bool miss = false;
#pragma unroll
                for (int u = 0; u < DF_U; u++) miss = miss || df_missing(xv[u]);
                if (!__ballot(miss) || !live) break;
                if (!df_backoff<DF_U>(a, spins, back, err)) {
                    live = false; // past the watchdog: the results are reported invalid
                    break;
                }
                df_poll<DF_U, true>(xv, col, x, k, rr);
            }
#pragma unroll
            for (int u = 0; u < DF_U; u++) acc = fma(v[u], xv[u], acc);
        }
        for (int o = kl; o < lanes; o <<= 1) acc += __shfl_xor(acc, o, WAVE);
        if (gq == 0 && mine) {
            double res = (b[(int64_t)ri.row * k + rr] - acc) / diag;
            if (df_missing(res)) res = __longlong_as_double(0x7FF8000000000000ll); // never: results are quiet
            cstore(x + (int64_t)ri.row * k + rr, res);
        }
    }
}

// The rows of one pass (df_pass): MIX, a mixed task whose row slots name their own codelets;
// otherwise the slots' tasks, whose codelet record, with one task per pass, is wave-uniform.
template <int KR, bool ADJ, bool VPERM, bool MIX>
__device__ __forceinline__ void df_rows(const SolveArgs &a, const Task &head, const Task &tk, DCod c, int t, int i,
                                        int lane) {
    constexpr int P = WAVE / KR, W = P / DF_RG;
    constexpr bool UNI = !MIX && W == 1;
    const int slot = lane / KR, r = lane % KR;
    int i0;
    bool active;
    if constexpr (MIX) {
        // a mixed task (one task per pass): row slot s is (codelet, row) slots[i0b + s]
        active = slot < head.i0e - head.i0b;
        const int2 sl = a.slots[head.i0b + (active ? slot : 0)];
        c = a.cods[sl.x];
        i0 = sl.y;
    } else {
        i0 = tk.i0b + i;
        active = t < a.ntasks && i0 < tk.i0e;
    }
    const MatInfo mi = mat_info(a, c);
    const int k = mi.k;
    const double *__restrict__ vals = a.vals + mi.val_base;
    const int32_t *__restrict__ perm = VPERM ? a.perm + mi.val_base : nullptr;
    const double *__restrict__ b = a.b + mi.vec_base;
    double *x = a.x + mi.vec_base;
    RowInfo ri{0, 0, 0};
    double diag = 1.0;
    if (active) {
        ri = row_info(c, a.aux, i0);
        const int dpos = ADJ ? ri.opst - 1 : ri.opst + ri.nops;
        diag = VPERM ? vals[perm[dpos]] : vals[dpos];
    }
    unsigned *err = a.err ? a.err : a.ctr + CTR_STRIDE;
    for (int r0 = 0; r0 < k; r0 += KR) { // more right-hand sides than lanes: KR = 8 only
        const int rr = r0 + r;
        const bool mine = active && rr < k; // this lane computes x[row, rr]
        const int nops = mine ? ri.nops : 0;
        const int64_t o = (int64_t)ri.row * k + rr;
        // ops in the order that leaves the latest dependences to the last chunk: ascending
        // columns for L, descending for U = L^T (its rows' first columns were solved last)
        ColIter<ADJ> it;
        it.mode = XM_STRIDED; // lanes without a row read no table
        it.base = 0;
        if (active) it.init(c, a.aux, i0, ri);
        // one task per pass and a rectangular codelet with a shared column table: every row has
        // nn ops, so an op's offset in the table is the same in every lane with a row and is read
        // with a scalar load
        const bool kshared = UNI && (c.flags & FRECT) && !(c.flags & DOPS) && xmode(c.flags) == XM_SHARED;
        const int cb = c.col0 + i0 * c.sigma0;
        const bool one_chunk = !__ballot(nops > DF_U);
        double acc = 0.0;
        bool pend = mine; // one chunk: the row's result is not stored yet
        for (int i1 = 0; __ballot(i1 < nops); i1 += DF_U) {
            double v[DF_U], xv[DF_U];
            int col[DF_U];
#pragma unroll
            for (int u = 0; u < DF_U; u++) {
                const bool ok = i1 + u < nops;
                const int op = ADJ ? nops - 1 - (i1 + u) : i1 + u;
                if (UNI && kshared) {
                    const int opu = min(ADJ ? c.nn - 1 - (i1 + u) : i1 + u, c.nn - 1);
                    const int xo = ((const_i32k_ptr)a.aux)[c.xt_off + max(opu, 0)];
                    col[u] = ok ? cb + xo : 0;
                } else {
                    col[u] = ok ? it.col(c, op) : 0;
                }
                const int e = ri.opst + op;
                v[u] = ok ? (VPERM ? vals[perm[e]] : vals[e]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < DF_U; u++) xv[u] = i1 + u < nops ? wload(x + (int64_t)col[u] * k + rr) : 0.0;
            const double bo = (one_chunk && mine) ? b[o] : 0.0;
            int64_t spins = 0;
            int back = 1;
            for (;;) {
                bool miss = false;
#pragma unroll
                for (int u = 0; u < DF_U; u++) miss = miss || df_missing(xv[u]);
                if (one_chunk) {
                    // a row whose values have all arrived is solved and stored at once, while
                    // the wave keeps waiting for its other rows
                    if (pend && !miss) {
                        df_finish<DF_U>(v, xv, acc, bo, diag, x + o);
                        pend = false;
                    }
                    if (!__ballot(pend)) break;
                } else if (!__ballot(miss)) {
                    break;
                }
                if (!df_backoff<DF_U>(a, spins, back, err)) {
                    // past the watchdog: the results are reported invalid, but every row is stored
                    if (one_chunk && pend) df_finish<DF_U>(v, xv, acc, bo, diag, x + o);
                    pend = false;
                    break;
                }
                df_poll<DF_U, (KR > 2)>(xv, col, x, k, rr);
            }
            if (!one_chunk) {
#pragma unroll
                for (int u = 0; u < DF_U; u++) acc = fma(v[u], xv[u], acc);
            }
        }
        // chunked rows, and rows of a pass whose rows have no ops at all (the chunk loop did not run)
        if (mine && (!one_chunk || pend)) {
            double res = (b[o] - acc) / diag;
            if (df_missing(res)) res = __longlong_as_double(0x7FF8000000000000ll); // never: results are quiet
            cstore(x + o, res);
        }
    }
}

// A mixed task's rows (batches) from their slot descriptors: a row's first value index,
// right-hand-side count, output element, ops and operand elements come from one 16-byte record
// and a list of absolute operand elements, instead of from its codelet record, its matrix's
// bases and the codelet's column tables, which shortens the pass's chain of dependent loads.
// A mixed row has at most DF_U ops, so its ops are one chunk.
constexpr int DF_MD_MASK = (1 << 27) - 1;

template <int KR, bool ADJ, bool VPERM>
__device__ __forceinline__ void df_mixed(const SolveArgs &a, const Task &head, int lane) {
    const int slot = lane / KR, r = lane % KR;
    const bool active = slot < head.i0e - head.i0b;
    const int4 d = a.mdesc[head.i0b + (active ? slot : 0)];
    const int e0 = d.x & DF_MD_MASK, k = (int)((unsigned)d.x >> 27) + 1;
    const int coff = d.z & DF_MD_MASK, rn = active ? (int)((unsigned)d.z >> 27) : 0;
    const int64_t rowel = d.y;
    const double *__restrict__ vals = a.vals + (VPERM ? d.w : 0);
    double diag = 1.0;
    if (active) {
        const int dpos = ADJ ? e0 - 1 : e0 + rn;
        diag = VPERM ? vals[a.perm[dpos]] : vals[dpos];
    }
    unsigned *err = a.err ? a.err : a.ctr + CTR_STRIDE;
    for (int r0 = 0; r0 < k; r0 += KR) { // a lane's own row sets k
        const int rr = r0 + r;
        const bool mine = active && rr < k;
        const int nops = mine ? rn : 0;
        const int64_t o = rowel + rr;
        double v[DF_U], xv[DF_U];
        int col[DF_U];
#pragma unroll
        for (int u = 0; u < DF_U; u++) {
            const bool ok = u < nops;
            const int op = ADJ ? nops - 1 - u : u;
            col[u] = ok ? a.mcols[coff + op] : 0;
            v[u] = ok ? (VPERM ? vals[a.perm[e0 + op]] : vals[e0 + op]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < DF_U; u++) xv[u] = u < nops ? wload(a.x + (int64_t)col[u] + rr) : 0.0;
        const double bo = mine ? a.b[o] : 0.0;
        int64_t spins = 0;
        int back = 1;
        bool pend = mine;
        for (;;) {
            bool miss = false;
#pragma unroll
            for (int u = 0; u < DF_U; u++) miss = miss || df_missing(xv[u]);
            if (pend && !miss) {
                df_finish<DF_U>(v, xv, 0.0, bo, diag, a.x + o);
                pend = false;
            }
            if (!__ballot(pend)) break;
            if (!df_backoff<DF_U>(a, spins, back, err)) {
                // past the watchdog: the results are reported invalid, but every row is stored
                if (pend) df_finish<DF_U>(v, xv, 0.0, bo, diag, a.x + o);
                pend = false;
                break;
            }
            df_poll<DF_U, (KR > 2)>(xv, col, a.x, 1, rr);
        }
    }
}

// One pass of a wave: rows of W consecutive tasks, KR lanes per row, lane r owning right-hand
// sides r, r + KR, ...  VPERM: the values through perm (the transposed solve reads L's values
// in U's order).  A pass whose first task is a wide-row task runs that task alone.
template <int KR, bool ADJ, bool VPERM>
__device__ __forceinline__ int df_pass(const SolveArgs &a, int p, int pn, int lane) {
    constexpr int P = WAVE / KR, W = P / DF_RG;
    const int slot = lane / KR, r = lane % KR;
    // the pass's first task, and each slot's task and codelet record, loaded together (before
    // the first task tells which kind of pass this is); and the same lines of the wave's next
    // pass (pn, when known), touched so that they are in the caches when it starts: the sum
    // returned keeps those loads
    // (pass indices are wave-uniform; with one task per pass, W = 1, so are the task's and the
    // touched next task's indices, and both are read through the constant address space: scalar
    // loads, served by the scalar cache)
    const int pu = __builtin_amdgcn_readfirstlane(p);
    const int t = pu * W + slot / DF_RG, i = slot % DF_RG;
    const int tc = W == 1 ? min(pu, a.ntasks - 1) : min(t, a.ntasks - 1);
    const Task head = k_task(a.tasks, pu * W);
    const Task tk = k_task(a.tasks, tc);
    DCod c = k_cod(a.tcods, tc);
    int touch = 0;
    if (pn >= 0 && pn < a.npass) {
        const int pnu = __builtin_amdgcn_readfirstlane(pn);
        const int tn = W == 1 ? min(pnu, a.ntasks - 1) : min(pnu * W + slot / DF_RG, a.ntasks - 1);
        touch = k_task(a.tasks, tn).meta + k_cod(a.tcods, tn).flags;
    }
    // a wide-row task runs alone; a pass that starts with an empty task is all empty (empty
    // tasks fill a group of DF_PASS_MAX up to its end)
    if (head.meta & DF_LONG) {
        df_long<ADJ, VPERM>(a, head, a.tcods[p * W], lane);
        return touch;
    }
    if (head.i0e == head.i0b) return touch;
    if (KR == DF_RG && (head.meta & DF_MIXED) && a.mdesc)
        df_mixed<KR, ADJ, VPERM>(a, head, lane);
    else if (KR == DF_RG && (head.meta & DF_MIXED))
        df_rows<KR, ADJ, VPERM, true>(a, head, tk, c, t, i, lane);
    else
        df_rows<KR, ADJ, VPERM, false>(a, head, tk, c, t, i, lane);
    return touch;
}

// ctr lines: 0 ticket, 1 error flag, 2 check-in count, 3 mode (0 undecided, 1 static, 2 ticket)
template <int KR, bool ADJ, bool VPERM>
__global__ __launch_bounds__(WAVE *WPB) void k_solve_df(SolveArgs a) {
    __shared__ int s_mode;
    unsigned *ticket = a.ctr, *arrive = a.ctr + 2 * CTR_STRIDE, *mode_w = a.ctr + 3 * CTR_STRIDE;
    if (threadIdx.x == 0) {
        const unsigned n = __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        unsigned want = 0u;
        if (n == gridDim.x) __hip_atomic_compare_exchange_strong(mode_w, &want, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
        unsigned m = cload_u(mode_w);
        for (int polls = 0; m == 0u; polls++) {
            if (polls >= DF_ARRIVE_POLLS) {
                want = 0u;
                __hip_atomic_compare_exchange_strong(mode_w, &want, 2u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
            }
            __builtin_amdgcn_s_sleep(8);
            m = cload_u(mode_w);
        }
        s_mode = (int)m;
    }
    __syncthreads();
    const int mode = s_mode;
    const int lane = threadIdx.x % WAVE;
    const unsigned one = lane == 0 ? 1u : 0u;
    const int nw = (int)gridDim.x * WPB;
    int p = mode == 1 ? (int)blockIdx.x * WPB + (int)threadIdx.x / WAVE
                      : __builtin_amdgcn_readfirstlane(
                            (int)__hip_atomic_fetch_add(ticket, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    int sink = 0;
    while (p < a.npass) {
        sink += df_pass<KR, ADJ, VPERM>(a, p, mode == 1 ? p + nw : -1, lane);
        p = mode == 1 ? p + nw
                      : __builtin_amdgcn_readfirstlane(
                            (int)__hip_atomic_fetch_add(ticket, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    // never true (npass >= 0): keeps the touch loads
    if (a.npass < 0 && sink == 1) a.x[0] = 0.0;
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < n; i += (int64_t)blockDim.x * gridDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------------------------------
// Single-block solve for matrices whose every level fits one pass of the block: one lane slot
// per (row, lane-of-row), levels separated by block barriers.
//
// One CU runs the whole solve, so a level costs a fixed latency (barrier, LDS round trips),
// the vector memory instructions its waves issue and the VALU issue of the waves that share a
// SIMD.  A lane fetches one stream entry per level (operand codes as LDS offsets, values over
// the diagonal) plus only the operands that must come from global memory; the others come
// from an LDS ring of the most recent solutions.  A wave's vector memory operations complete
// in issue order, so nothing on a level's critical path reads global memory: the stream entry
// is fetched four levels ahead and the global operands (rows final by then) two levels ahead.
// Helper blocks dispatched to the solver's XCD pull the stream and the global operands of the
// levels just ahead into the shared L2.
// ------------------------------------------------------------------------------------------

// Lane exchange within 16-lane rows through DPP (no LDS round trip): the value of lane
// i ^ d for d in {1, 2, 4, 8}; other distances go through the LDS crossbar.
// DPP moves with every source lane valid where the result is used (bound_ctrl set, so that no
// old value has to be kept in the destination)
template <int D> __device__ __forceinline__ int dpp_xor_i(int v) {
    if constexpr (D == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);      // quad_perm 1,0,3,2
    else if constexpr (D == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true); // quad_perm 2,3,0,1
    else if constexpr (D == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true); // row_ror 8
    else {
        const int up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0xF, true); // row_shl 4: lane i + 4
        const int dn = __builtin_amdgcn_mov_dpp(v, 0x114, 0xF, 0xF, true); // row_shr 4: lane i - 4
        return (__lane_id() & 4) ? dn : up;
    }
}
template <int D> __device__ __forceinline__ double dpp_xor(double v) {
    const int lo = dpp_xor_i<D>(__double2loint(v)), hi = dpp_xor_i<D>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
// v of lane i ^ D: DPP within 16-lane rows for D <= 8, the LDS crossbar beyond
template <int D> __device__ __forceinline__ double lane_xor(double v) {
    if constexpr (D <= 8) return dpp_xor<D>(v);
    else return __shfl_xor(v, D, WAVE);
}
// sum over aligned groups of G = 2^LG lanes; every lane gets its group's sum
template <int LG, int KT> __device__ __forceinline__ void group_sum_c(double (&acc)[KT]) {
    if constexpr (LG > 0) {
        group_sum_c<LG - 1, KT>(acc);
#pragma unroll
        for (int r = 0; r < KT; r++) acc[r] += lane_xor<(1 << (LG - 1))>(acc[r]);
    }
}

// level table entry through the constant address space: a scalar load, counted apart from the
// vector memory operations
typedef const __attribute__((address_space(4))) long long *const_i64_ptr;
__device__ __forceinline__ int4 thin_lvl(const ThinArgs &a, int l) {
    const const_i64_ptr p = (const_i64_ptr)(a.lvl) + 2 * (int64_t)l;
    const long long e0 = p[0], e1 = p[1];
    return make_int4((int)(unsigned)(e0 & 0xffffffffll), (int)(e0 >> 32), (int)(unsigned)(e1 & 0xffffffffll),
                     (int)(e1 >> 32));
}

template <int KT> struct ThinA {
    int code[THIN_SLOTS];
    double v[THIN_SLOTS]; // values over the diagonal
    int pin;              // the writer's second LDS entry (byte offset)
};
template <int KT, int NGS> struct ThinB {
    double gx[NGS > 0 ? NGS : 1][KT]; // operands gathered from global memory
};

// Fetches are issued by every wave, also one with no record at the level (it reads the
// stream's chunk of empty records, which stays in the L1 cache): a fetch on one path only
// would make the compiler's wait counts cover it on both.
template <int KT>
__device__ __forceinline__ void thin_fetch_a(const ThinArgs &a, int l, int s, ThinA<KT> &t) {
    const int4 lv = thin_lvl(a, l);
    // the wave's chunk of 64 records (a level's records start on a chunk), or the empty chunk
    // for a wave with no record at the level; lanes past the level's records read placeholders
    const int wv = __builtin_amdgcn_readfirstlane(s / WAVE);
    const int64_t chunk = wv * WAVE < lv.y ? (int64_t)(lv.x / WAVE) + wv : a.n_rec / WAVE;
    const double *w = a.stream + chunk * (64 * THIN_SW) + (s & (WAVE - 1)) * 2;
    const int4 c = *reinterpret_cast<const int4 *>(w);
    const double2 v01 = *reinterpret_cast<const double2 *>(w + 128);
    const double2 v23 = *reinterpret_cast<const double2 *>(w + 256);
    const int4 v4c = *reinterpret_cast<const int4 *>(w + 384);
    t.code[0] = c.x; t.code[1] = c.y; t.code[2] = c.z; t.code[3] = c.w;
    t.code[4] = v4c.z;
    t.pin = v4c.w;
    t.v[0] = v01.x; t.v[1] = v01.y; t.v[2] = v23.x; t.v[3] = v23.y;
    t.v[4] = __hiloint2double(v4c.y, v4c.x);
    static_assert(KT == 1, "one right-hand side");
}

template <int KT, int NGS>
__device__ __forceinline__ void thin_fetch_b(const ThinArgs &a, const ThinA<KT> &t, ThinB<KT, NGS> &u) {
    static_assert(KT == 1, "one right-hand side");
#pragma unroll
    for (int j = 0; j < NGS; j++) {
        // a global operand -(1 + solve-order index); any other code reads the zero past the
        // solutions
        const int c = t.code[j];
        u.gx[j][0] = a.xs[c < 0 ? ~c : a.n];
    }
}

template <int KT, int NGS, int LG, bool PIN>
__device__ __forceinline__ void thin_compute(const ThinArgs &a, int l, int s, const ThinA<KT> &t,
                                             const ThinB<KT, NGS> &u, double *ring) {
    constexpr int G = 1 << LG;
    const int g = s & (G - 1);
    const int4 lv = thin_lvl(a, l);
    double acc[KT];
#pragma unroll
    for (int rr = 0; rr < KT; rr++) acc[rr] = 0.0;
    const char *lds = reinterpret_cast<const char *>(ring);
#pragma unroll
    for (int j = 0; j < THIN_SLOTS; j++) {
        // the code is the operand's byte offset in LDS; in the first NGS slots a negative code
        // is a global operand (gathered, while the LDS read takes the zero entry)
        const int c = t.code[j];
        const int off = (j < NGS && c < 0) ? (a.ring + 1) * 8 : c;
        double xo = *reinterpret_cast<const double *>(lds + off);
        if (j < NGS) xo += u.gx[j < NGS ? j : 0][0];
        acc[0] = fma(t.v[j], xo, acc[0]);
    }
    group_sum_c<LG, KT>(acc);
    // lanes below ww hold the level's rows of 2G lanes (the level table counts them)
    const int ww = lv.w << (LG + 1);
    if (lv.w > 0) {
        // rows of 2G lanes: add the other half
#pragma unroll
        for (int rr = 0; rr < KT; rr++) {
            const double o = lane_xor<G>(acc[rr]);
            if (s < ww) acc[rr] += o;
        }
    }
    if (s < lv.y && (s >= ww || !(s & G))) {
        // solve-order index: the level's first, plus the row's rank (wide rows of 2G lanes first)
        const int64_t rp = lv.z + (s < ww ? s >> (LG + 1) : lv.w + ((s - ww) >> LG));
        const int slot = (int)(rp & (a.ring - 1));
#pragma unroll
        for (int rr = 0; rr < KT; rr++)
            if ((rr & (G - 1)) == g) { // one right-hand side per call
                const double xn = -acc[rr]; // the slots sum to -(b - sum of ops) / diagonal
                a.xs[rp * KT + rr] = xn;
                ring[slot * KT + rr] = xn;
                if constexpr (PIN) *reinterpret_cast<double *>(reinterpret_cast<char *>(ring) + t.pin) = xn;
            }
    }
}

// One level: solve it, then gather the global operands of the level two ahead and fetch the
// stream entry of the level four ahead (into the slot this level used).
template <int KT, int NGS, int LG, bool PIN>
__device__ __forceinline__ void thin_step(const ThinArgs &a, int l, int s, ThinA<KT> &a0, ThinB<KT, NGS> &b0,
                                          const ThinA<KT> &a2, double *ring) {
    thin_compute<KT, NGS, LG, PIN>(a, l, s, a0, b0, ring);
    __builtin_amdgcn_sched_barrier(0);
    thin_fetch_b<KT, NGS>(a, a2, b0);
    thin_fetch_a<KT>(a, l + 4, s, a0);
    __builtin_amdgcn_sched_barrier(0);
    if (s == 0 && (l & 3) == 3)
        __hip_atomic_store(a.progress, (unsigned)(l + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
}

// Helper blocks: each wave takes every nw-th level and touches each 128-byte line of its
// stream entries and of its global operands, staying at most `ahead` levels in front of the
// solver.  A helper that waits
// past its poll limit just stops (the solver never waits for it).
__device__ void thin_helper(const ThinArgs &a) {
    const int h = (int)blockIdx.x / 8 - 1;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int wpb = (int)blockDim.x / WAVE, nw = a.helpers * wpb;
    unsigned sink = 0;
    int seen = 0;
    int64_t polls = 0;
    for (int l = 3 + h * wpb + wave; l < a.nlev; l += nw) {
        while (seen + a.ahead < l) {
            seen = __builtin_amdgcn_readfirstlane((int)cload_u(a.progress));
            if (seen + a.ahead >= l) break;
            if (++polls > (int64_t(1) << 24)) return;
            __builtin_amdgcn_s_sleep(4);
        }
        const int4 lv = thin_lvl(a, l);
        const uintptr_t s0 = reinterpret_cast<uintptr_t>(a.stream + (int64_t)lv.x * THIN_SW);
        const uintptr_t s1 = s0 + (uintptr_t)((lv.y + 63) & ~63) * THIN_SW * 8;
#pragma unroll 4
        for (uintptr_t o = (s0 & ~uintptr_t(127)) + lane * 128; o < s1; o += WAVE * 128)
            sink ^= *reinterpret_cast<const unsigned *>(o);
        // and the lines of the solutions its global operands read (rows solved long before,
        // mostly out of the L2 cache by now); a line touched before its row is solved is
        // only brought in early
        for (int r = lane; r < lv.y; r += WAVE) {
            const int64_t p = (int64_t)lv.x + r;
            const double *w = a.stream + (p >> 6) * (64 * THIN_SW) + (p & 63) * 2;
            // global operands sit in the first ngs slots, coded -(1 + solve-order index)
            const int4 c = *reinterpret_cast<const int4 *>(w);
            const int c4 = reinterpret_cast<const int *>(w + 384)[2];
            if (c.x < 0 && a.ngs > 0) sink ^= *reinterpret_cast<const unsigned *>(a.xs + ~c.x);
            if (c.y < 0 && a.ngs > 1) sink ^= *reinterpret_cast<const unsigned *>(a.xs + ~c.y);
            if (c.z < 0 && a.ngs > 2) sink ^= *reinterpret_cast<const unsigned *>(a.xs + ~c.z);
            if (c.w < 0 && a.ngs > 3) sink ^= *reinterpret_cast<const unsigned *>(a.xs + ~c.w);
            if (c4 < 0 && a.ngs > 4) sink ^= *reinterpret_cast<const unsigned *>(a.xs + ~c4);
        }
    }
    if (sink == 0x9e3779b9u) *a.sink = sink; // keeps the loads
}

template <int KT, int NGS, int LG, bool PIN>
__global__ __launch_bounds__(THIN_THREADS) void k_solve_thin(ThinArgs a) {
    static_assert(THIN_SLOTS == 5, "stream layout");
    if (blockIdx.x != 0) {
        // blocks are dispatched round robin over the 8 XCDs: multiples of 8 share block 0's L2
        if (blockIdx.x % 8 == 0) thin_helper(a);
        return;
    }
    // the ring at a fixed LDS address (no base to add to each operand's offset), sized for the
    // largest ring, then the -1 and 0 entries and the pinned entries (after the plan's ring)
    __shared__ double ring[THIN_RING_MAX + 2 + THIN_PIN];
    const int s = threadIdx.x;
    if (s == 0) {
        ring[a.ring] = -1.0;    // operand of the right-hand-side terms
        ring[a.ring + 1] = 0.0; // operand of empty slots
    }
    __syncthreads();
    ThinA<KT> A0, A1, A2, A3;
    ThinB<KT, NGS> B0, B1;
    // same issue order as the loop's steady state (gathers for l + 1, then stream l + 3), so
    // the compiler's wait counts at the loop head agree on both entries
    thin_fetch_a<KT>(a, 0, s, A0);
    thin_fetch_a<KT>(a, 1, s, A1);
    __builtin_amdgcn_sched_barrier(0);
    thin_fetch_b<KT, NGS>(a, A0, B0);
    thin_fetch_a<KT>(a, 2, s, A2);
    __builtin_amdgcn_sched_barrier(0);
    thin_fetch_b<KT, NGS>(a, A1, B1);
    thin_fetch_a<KT>(a, 3, s, A3);
    __builtin_amdgcn_sched_barrier(0);
    for (int l = 0; l < a.nlev_pad; l += 4) {
        thin_step<KT, NGS, LG, PIN>(a, l, s, A0, B0, A2, ring);
        thin_step<KT, NGS, LG, PIN>(a, l + 1, s, A1, B1, A3, ring);
        thin_step<KT, NGS, LG, PIN>(a, l + 2, s, A2, B0, A0, ring);
        thin_step<KT, NGS, LG, PIN>(a, l + 3, s, A3, B1, A1, ring);
    }
}

// Once per upload: each slot's stream code (an LDS byte offset, or a global operand), and the
// chunk of empty records, codes and values.
__global__ __launch_bounds__(256) void k_thin_codes(ThinArgs a) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n_rec + 64) return;
    double *w = a.stream + (p >> 6) * (64 * THIN_SW) + (p & 63) * 2;
    const int zero = (a.ring + 1) * 8; // LDS byte offset of the zero entry
    if (p >= a.n_rec) {
        // the chunk of empty records
        *reinterpret_cast<int4 *>(w) = make_int4(zero, zero, zero, zero);
        *reinterpret_cast<double2 *>(w + 128) = make_double2(0.0, 0.0);
        *reinterpret_cast<double2 *>(w + 256) = make_double2(0.0, 0.0);
        *reinterpret_cast<int4 *>(w + 384) = make_int4(0, 0, zero, 0);
        return;
    }
    static_assert(THIN_REC == 21 && THIN_SLOTS == 5, "record layout");
    const int32_t *co = a.rec + p * THIN_REC + 4 + 2 * THIN_SLOTS;
    const int pin = a.rec[p * THIN_REC + THIN_REC - 1]; // the writer's second LDS entry
    int code[THIN_SLOTS];
#pragma unroll
    for (int j = 0; j < THIN_SLOTS; j++) {
        // table codes: >= 0 global solve-order index, THIN_UNUSED empty, else -(1 + LDS entry)
        const int c = co[j];
        code[j] = c >= 0 ? ~c : c == THIN_UNUSED ? zero : ~c * 8;
    }
    *reinterpret_cast<int4 *>(w) = make_int4(code[0], code[1], code[2], code[3]);
    *reinterpret_cast<int2 *>(w + 385) = make_int2(code[4], pin < 0 ? 0 : pin * 8);
}

// Per call, in record order: each slot's value over the row's diagonal (0 for empty slots, b
// for the right-hand-side term); the codes stay.  Also clears the solver's progress word.
__global__ __launch_bounds__(256) void k_thin_stream(ThinArgs a) {
    const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x, a.remap) * 256 + threadIdx.x;
    if (p == 0) {
        *a.progress = 0u;
        a.xs[a.n] = 0.0; // read by gathers of slots without a global operand
    }
    if (p >= a.n_rec) return;
    const int32_t *g = a.gidx + (p >> 6) * (64 * THIN_GIDX);
    const int4 g4 = reinterpret_cast<const int4 *>(g)[p & 63];
    const int2 g2 = reinterpret_cast<const int2 *>(g + 64 * 4)[p & 63];
    const int32_t vi[THIN_SLOTS] = {g4.x, g4.y, g4.z, g4.w, g2.x};
    const double d = a.vals[g2.y];
    double v[THIN_SLOTS];
#pragma unroll
    for (int j = 0; j < THIN_SLOTS; j++) {
        const int32_t i = vi[j];
        v[j] = i == THIN_UNUSED ? 0.0 : (i < 0 ? a.b[(int64_t)(-2 - i) * a.k] : a.vals[i]) / d;
    }
    double *w = a.stream + (p >> 6) * (64 * THIN_SW) + (p & 63) * 2;
    *reinterpret_cast<double2 *>(w + 128) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2 *>(w + 256) = make_double2(v[2], v[3]);
    w[384] = v[4];
}

// Solutions from solve order into row order.
__global__ __launch_bounds__(256) void k_thin_scatter(ThinArgs a) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= a.n) return;
    const int64_t row = a.rows[q];
    for (int r = 0; r < a.k; r++) a.x[row * a.k + r] = a.xs[q * a.kt + r];
}

__global__ void k_reset(unsigned *p, int64_t n) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < n; i += (int64_t)blockDim.x * gridDim.x)
        p[i] = 0u;
}

__global__ void k_fill(double *p, int64_t n, double v) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < n; i += (int64_t)blockDim.x * gridDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------------------------------
// Plain comparators: CSR with G lanes per row, no codelets.
// ------------------------------------------------------------------------------------------
template <int KT>
__global__ __launch_bounds__(WAVE *WPB) void k_csr_spmv(PlainArgs a) {
    const int lane = threadIdx.x % WAVE;
    const int lg = a.lg, G = 1 << lg, R = WAVE >> lg;
    const int64_t row = ((int64_t)blockIdx.x * WPB + threadIdx.x / WAVE) * R + (lane >> lg);
    const int g = lane & (G - 1);
    const bool active = row < a.n;
    const int k = a.k;
    const int b = active ? a.rp[row] : 0, e1 = active ? a.rp[row + 1] : 0;
    for (int r0 = 0; r0 < k; r0 += KT) {
        double acc[KT];
#pragma unroll
        for (int r = 0; r < KT; r++) acc[r] = 0.0;
        for (int e = b + g; e < e1; e += G) {
            const double v = a.vals[e];
            const double *__restrict__ xr = a.x + (int64_t)a.ci[e] * k + r0;
#pragma unroll
            for (int r = 0; r < KT; r++)
                if (r0 + r < k) acc[r] += v * xr[r];
        }
        group_sum<KT>(acc, G);
        if (active) {
#pragma unroll
            for (int r = 0; r < KT; r++)
                if ((r & (G - 1)) == g && r0 + r < k) a.y[row * k + r0 + r] = acc[r];
        }
    }
}

// one level of the solve: rows rows[lo..hi); upper = 1 reads U = L^T (diagonal first,
// values through perm), else L (diagonal last)
template <int KT>
__global__ __launch_bounds__(WAVE *WPB) void k_csr_level(PlainArgs a) {
    const int lane = threadIdx.x % WAVE;
    const int lg = a.lg, G = 1 << lg, R = WAVE >> lg;
    const int64_t p = a.lo + ((int64_t)blockIdx.x * WPB + threadIdx.x / WAVE) * R + (lane >> lg);
    const int g = lane & (G - 1);
    const bool active = p < a.hi;
    const int k = a.k;
    const int64_t row = active ? a.rows[p] : 0;
    int b = 0, e1 = 0, d = 0;
    double diag = 1.0;
    if (active) {
        b = a.rp[row];
        e1 = a.rp[row + 1];
        if (a.upper) {
            d = b;
            b += 1;
        } else {
            d = e1 - 1;
            e1 -= 1;
        }
        diag = a.upper ? a.vals[a.perm[d]] : a.vals[d];
    }
    for (int r0 = 0; r0 < k; r0 += KT) {
        double acc[KT];
#pragma unroll
        for (int r = 0; r < KT; r++) acc[r] = 0.0;
        for (int e = b + g; e < e1; e += G) {
            const double v = a.upper ? a.vals[a.perm[e]] : a.vals[e];
            const double *__restrict__ xr = a.y + (int64_t)a.ci[e] * k + r0;
#pragma unroll
            for (int r = 0; r < KT; r++)
                if (r0 + r < k) acc[r] += v * xr[r];
        }
        group_sum<KT>(acc, G);
        if (active) {
#pragma unroll
            for (int r = 0; r < KT; r++)
                if ((r & (G - 1)) == g && r0 + r < k)
                    a.y[row * k + r0 + r] = (a.x[row * k + r0 + r] - acc[r]) / diag;
        }
    }
}

// SpMV adjoint with FP64 atomics: GX[col] += v g[row]; GV[e] = sum_r g[row, r] x[col, r]
__global__ __launch_bounds__(WAVE *WPB) void k_csr_spmv_adj_atomic(PlainArgs a) {
    const int lane = threadIdx.x % WAVE;
    const int lg = a.lg, G = 1 << lg, R = WAVE >> lg;
    const int64_t row = ((int64_t)blockIdx.x * WPB + threadIdx.x / WAVE) * R + (lane >> lg);
    const int g = lane & (G - 1);
    if (row >= a.n) return;
    const int k = a.k;
    const double *__restrict__ gr = a.g + row * k;
    for (int e = a.rp[row] + g; e < a.rp[row + 1]; e += G) {
        const int64_t c = a.ci[e];
        const double v = a.vals[e];
        double s = 0.0;
        for (int r = 0; r < k; r++) {
            s += gr[r] * a.x[c * k + r];
            if (a.y) atomicAdd(a.y + c * k + r, v * gr[r]);
        }
        if (a.gv) a.gv[e] = s;
    }
}

// GV of the solve adjoint over L's CSR: gv[e] = -sum_r lam[row, r] x[col, r]
__global__ __launch_bounds__(WAVE *WPB) void k_csr_gv(PlainArgs a) {
    const int lane = threadIdx.x % WAVE;
    const int lg = a.lg, G = 1 << lg, R = WAVE >> lg;
    const int64_t row = ((int64_t)blockIdx.x * WPB + threadIdx.x / WAVE) * R + (lane >> lg);
    const int g = lane & (G - 1);
    if (row >= a.n) return;
    const int k = a.k;
    const double *__restrict__ lr = a.g + row * k;
    for (int e = a.rp[row] + g; e < a.rp[row + 1]; e += G) {
        const int64_t c = a.ci[e];
        double s = 0.0;
        for (int r = 0; r < k; r++) s += lr[r] * a.x[c * k + r];
        a.gv[e] = -s;
    }
}

// Value gradient of an adjoint (GvArgs): G lanes per row, each lane one entry at a time; the
// row of g in registers; x rows read whole (16-byte loads when VEC: k even, 16-byte aligned
// vectors).  Any k up to KT (a power of two): slots past k are predicated off (EXACT: k = KT,
// no predicates).
template <int KT, bool EXACT>
__device__ __forceinline__ void gv_row_load(const double *__restrict__ gr, int k, double (&gw)[KT]) {
#pragma unroll
    for (int r = 0; r < KT; r++) gw[r] = (EXACT || r < k) ? gr[r] : 0.0;
}

template <int KT, bool VEC, bool EXACT>
__device__ __forceinline__ double gv_dot(const double (&gw)[KT], const double *__restrict__ xr, int k) {
    double s = 0.0;
    if constexpr (VEC) {
#pragma unroll
        for (int r = 0; r < KT; r += 2)
            if (EXACT || r < k) {
                const double2 q = *reinterpret_cast<const double2 *>(xr + r);
                s = fma(gw[r], q.x, s);
                s = fma(gw[r + 1], q.y, s);
            }
    } else {
#pragma unroll
        for (int r = 0; r < KT; r++)
            if (EXACT || r < k) s = fma(gw[r], xr[r], s);
    }
    return s;
}

template <int KT, bool VEC, bool EXACT> __global__ __launch_bounds__(WAVE *WPB) void k_gv_csr(GvArgs a) {
    const int lane = threadIdx.x % WAVE;
    const int lg = a.lg, G = 1 << lg, R = WAVE >> lg;
    const int64_t row = ((int64_t)blockIdx.x * WPB + threadIdx.x / WAVE) * R + (lane >> lg);
    const int g = lane & (G - 1);
    if (row >= a.n) return;
    const int k = a.k;
    const int e1 = a.rp[row + 1];
    if (e1 - a.rp[row] > GV_LONG_ROW) return; // in the chunk pass
    double gw[KT];
    gv_row_load<KT, EXACT>(a.g + row * k, k, gw);
    for (int e = a.rp[row] + g; e < e1; e += G) a.gv[e] = a.sign * gv_dot<KT, VEC, EXACT>(gw, a.x + (int64_t)a.ci[e] * k, k);
}

// The chunks of long rows: a wave per GV_CHUNK entries of one row, 8 entries a lane.
template <int KT, bool VEC, bool EXACT> __global__ __launch_bounds__(WAVE *WPB) void k_gv_chunks(GvArgs a) {
    const int64_t c = (int64_t)blockIdx.x * WPB + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (c >= a.n_chunks) return;
    const int2 ch = a.chunks[c];
    const int64_t row = ch.x;
    const int k = a.k;
    double gw[KT];
    gv_row_load<KT, EXACT>(a.g + row * k, k, gw);
    const int e1 = min(a.rp[row + 1], ch.y + GV_CHUNK);
    for (int e = ch.y + lane; e < e1; e += WAVE) a.gv[e] = a.sign * gv_dot<KT, VEC, EXACT>(gw, a.x + (int64_t)a.ci[e] * k, k);
}

// The SpMV adjoint's value gradient through the forward plan's several-right-hand-side tasks:
// GV[e] = sign * sum_r G[row, r] X[col, r] for every op e of every codelet (in the forward plan
// an op's index is its value index).  The lane layout is k_spmvN's: KR lanes per row, RV
// consecutive right-hand sides per lane, so the x rows of P consecutive rows are read as
// contiguous 16-byte pieces across the wave, and the KR lanes of a row add their partial dots
// by cross-lane exchange.  Rectangular codelets with row-major contiguous ops collect their P
// rows' gradients in LDS and write them with coalesced stores; other codelets write each op's
// gradient from the row's first lane.  Rows of a wave past the task's end repeat its last row
// (same values, no stores), which keeps every lane of the exchange active.
template <int KR> __device__ __forceinline__ double kr_sum(double s) {
    if constexpr (KR >= 2) s += lane_xor<1>(s);
    if constexpr (KR >= 4) s += lane_xor<2>(s);
    if constexpr (KR >= 8) s += lane_xor<4>(s);
    if constexpr (KR >= 16) s += lane_xor<8>(s);
    return s;
}

template <int RV>
__device__ __forceinline__ double rv_dot(const double (&gw)[RV], const double *__restrict__ xr) {
    double s = 0.0;
#pragma unroll
    for (int h = 0; h < RV / 2; h++) {
        const double2 q = reinterpret_cast<const double2 *>(xr)[h];
        s = fma(gw[2 * h], q.x, s);
        s = fma(gw[2 * h + 1], q.y, s);
    }
    return s;
}

template <int RV> __device__ __forceinline__ void rv_load(const double *__restrict__ gr, double (&gw)[RV]) {
#pragma unroll
    for (int h = 0; h < RV / 2; h++) {
        const double2 q = reinterpret_cast<const double2 *>(gr)[h];
        gw[2 * h] = q.x;
        gw[2 * h + 1] = q.y;
    }
}

template <int KR, int RV, int MODE, bool STG>
__device__ __forceinline__ void gv_rect(const GvPlanArgs &a, const DCod &c, const Task &tk, int lane, double *sv) {
    constexpr int P = WAVE / KR;
    const int slot = lane / KR, r = (lane % KR) * RV;
    const int k = a.k, nn = c.nn;
    for (int base = tk.i0b; base < tk.i0e; base += P) {
        const int i0 = min(base + slot, tk.i0e - 1);
        const bool active = base + slot < tk.i0e;
        const int row = row_of(c, a.aux, i0);
        const int opst = c.op0 + i0 * c.op_step;
        const int cbase = (MODE == XM_FULL) ? c.xt_off + i0 * nn : c.col0 + i0 * c.sigma0;
        double gw[RV];
        rv_load<RV>(a.g + (int64_t)row * k + r, gw);
        for (int i1 = 0; i1 < nn; i1 += RUV) {
            int col[RUV];
            double2 xv[RUV][RV / 2];
#pragma unroll
            for (int u = 0; u < RUV; u++) {
                const int j = min(i1 + u, nn - 1);
                if constexpr (MODE == XM_STRIDED)
                    col[u] = cbase + j * c.sigma1;
                else if constexpr (MODE == XM_SHARED)
                    col[u] = cbase + ((const_i32k_ptr)a.aux)[c.xt_off + j];
                else
                    col[u] = a.aux[cbase + j];
            }
#pragma unroll
            for (int u = 0; u < RUV; u++) {
                const double2 *xp = reinterpret_cast<const double2 *>(a.x + (int64_t)col[u] * k + r);
#pragma unroll
                for (int h = 0; h < RV / 2; h++) xv[u][h] = xp[h];
            }
#pragma unroll
            for (int u = 0; u < RUV; u++) {
                double d = 0.0;
#pragma unroll
                for (int h = 0; h < RV / 2; h++) {
                    d = fma(gw[2 * h], xv[u][h].x, d);
                    d = fma(gw[2 * h + 1], xv[u][h].y, d);
                }
                d = a.sign * kr_sum<KR>(d);
                if (i1 + u < nn && r == 0) {
                    if constexpr (STG)
                        sv[(i0 - base) * nn + i1 + u] = d;
                    else if (active)
                        a.gv[opst + i1 + u] = d;
                }
            }
        }
        if constexpr (STG) {
            wave_sync();
            const int e0 = c.op0 + base * nn, ne = min(P, tk.i0e - base) * nn;
            for (int q = lane; q < ne; q += WAVE) a.gv[e0 + q] = sv[q];
            wave_sync();
        }
    }
}

template <int KR, int RV>
__device__ __forceinline__ void gv_walk(const GvPlanArgs &a, const DCod &c, const Task &tk, int lane) {
    constexpr int P = WAVE / KR;
    const int slot = lane / KR, r = (lane % KR) * RV;
    const int k = a.k;
    const int mode = xmode(c.flags);
    for (int base = tk.i0b; base < tk.i0e; base += P) {
        const int i0 = min(base + slot, tk.i0e - 1);
        const bool active = base + slot < tk.i0e;
        const RowInfo ri = row_info(c, a.aux, i0);
        double gw[RV];
        rv_load<RV>(a.g + (int64_t)ri.row * k + r, gw);
        walk_any(mode, c, a.aux, i0, ri, 0, 1, [&](int e, int col) {
            const double d = a.sign * kr_sum<KR>(rv_dot<RV>(gw, a.x + (int64_t)col * k + r));
            if (active && r == 0) a.gv[e] = d;
        });
    }
}

template <int KR, int RV> __global__ __launch_bounds__(WAVE *WPB, 4) void k_gv_plan(GvPlanArgs a) {
    __shared__ double sv_all[WPB][SV_CAP];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int t = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x, a.remap) * WPB + wave);
    if (t >= a.ntasks) return;
    const Task tk = k_task(a.tasks, t);
    const DCod c = k_cod(a.cods, tk.cod);
    const int mode = xmode(c.flags);
    const bool rect = (c.flags & FRECT) && !(c.flags & DOPS) && c.nn > 0;
    const bool stg = c.op_step == c.nn && (WAVE / KR) * c.nn <= SV_CAP;
    double *sv = sv_all[wave];
    if (rect && stg && mode == XM_SHARED)
        gv_rect<KR, RV, XM_SHARED, true>(a, c, tk, lane, sv);
    else if (rect && stg && mode == XM_STRIDED)
        gv_rect<KR, RV, XM_STRIDED, true>(a, c, tk, lane, sv);
    else if (rect && stg && mode == XM_FULL)
        gv_rect<KR, RV, XM_FULL, true>(a, c, tk, lane, sv);
    else if (rect && mode == XM_SHARED)
        gv_rect<KR, RV, XM_SHARED, false>(a, c, tk, lane, sv);
    else if (rect && mode == XM_STRIDED)
        gv_rect<KR, RV, XM_STRIDED, false>(a, c, tk, lane, sv);
    else if (rect && mode == XM_FULL)
        gv_rect<KR, RV, XM_FULL, false>(a, c, tk, lane, sv);
    else
        gv_walk<KR, RV>(a, c, tk, lane);
}

// One entry's value gradient in a batch: k of the matrix (at most KT) decides the predicates
// and the vector loads at run time (matrices of one class differ).
template <int KT>
__device__ __forceinline__ double gv_dot_any(const double (&gw)[KT], const double *__restrict__ xr, int k, bool vec) {
    if constexpr (KT == 1) {
        return gv_dot<1, false, true>(gw, xr, k);
    } else {
        if (k == KT) return vec ? gv_dot<KT, true, true>(gw, xr, k) : gv_dot<KT, false, true>(gw, xr, k);
        return vec ? gv_dot<KT, true, false>(gw, xr, k) : gv_dot<KT, false, false>(gw, xr, k);
    }
}

// Matrix of row q of a class (binary search over the class's row starts).
__device__ __forceinline__ int gv_class_mat(const GvBatchArgs &a, int64_t q) {
    int lo = 0, hi = a.nm - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.mstart[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int KT> __global__ __launch_bounds__(WAVE *WPB) void k_gv_batch(GvBatchArgs a) {
    const int lane = threadIdx.x % WAVE;
    const int lg = a.lg, G = 1 << lg, R = WAVE >> lg;
    const int64_t q = ((int64_t)blockIdx.x * WPB + threadIdx.x / WAVE) * R + (lane >> lg);
    const int g = lane & (G - 1);
    if (q >= a.n) return;
    const int j = gv_class_mat(a, q);
    const MatInfo mi = a.mats[a.mids[j]];
    const int64_t row = q - a.mstart[j];
    const int k = mi.k;
    const int32_t *__restrict__ rp = a.rp + mi.row_base;
    const int e1 = rp[row + 1];
    if (e1 - rp[row] > GV_LONG_ROW) return; // in the chunk pass
    const bool vec = a.aligned && k % 2 == 0 && mi.vec_base % 2 == 0;
    double gw[KT];
    if (k == KT) gv_row_load<KT, true>(a.g + mi.vec_base + row * k, k, gw);
    else gv_row_load<KT, false>(a.g + mi.vec_base + row * k, k, gw);
    const double *__restrict__ x = a.x + mi.vec_base;
    for (int e = rp[row] + g; e < e1; e += G) a.gv[e] = -gv_dot_any<KT>(gw, x + (int64_t)a.ci[e] * k, k, vec);
}

// The chunks of a class's long rows: a wave per GV_CHUNK entries of one row.
template <int KT> __global__ __launch_bounds__(WAVE *WPB) void k_gv_batch_chunks(GvBatchArgs a) {
    const int64_t c = (int64_t)blockIdx.x * WPB + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (c >= a.n_chunks) return;
    const int4 ch = a.chunks[c];
    const MatInfo mi = a.mats[ch.x];
    const int64_t row = ch.y;
    const int k = mi.k;
    const bool vec = a.aligned && k % 2 == 0 && mi.vec_base % 2 == 0;
    double gw[KT];
    if (k == KT) gv_row_load<KT, true>(a.g + mi.vec_base + row * k, k, gw);
    else gv_row_load<KT, false>(a.g + mi.vec_base + row * k, k, gw);
    const double *__restrict__ x = a.x + mi.vec_base;
    const int e1 = min(a.rp[mi.row_base + row + 1], ch.z + GV_CHUNK);
    for (int e = ch.z + lane; e < e1; e += WAVE) a.gv[e] = -gv_dot_any<KT>(gw, x + (int64_t)a.ci[e] * k, k, vec);
}

// Column-slice (BLAS-only) plans.  Every codelet is ops [a, a + nn) of m rows with all three
// access functions strided, so a row's ops may lie in several codelets: each task's rows add
// their slice's partial sums into the row (SpMV: into y; solve: into the row's accumulator), one
// FP64 atomic add per row and right-hand side.  KR == 1 (one right-hand side): G lanes to a row
// (G from the task) with a shuffle reduction; KR > 1: KR lanes to a row, lane r owning
// right-hand sides r, r + KR, ...  In the solve every contributing lane then counts itself into
// the row's tally after a device-scope fence, and the lane whose count completes the tally
// (slices x contributing lanes per slice) reads the sums back from L2 and writes the solution.
template <bool SOLVE, int KR> __global__ __launch_bounds__(WAVE *WPB) void k_slices(SliceArgs a) {
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int t = blockIdx.x * WPB + wave;
    if (t >= a.ntasks) return;
    const Task tk = a.tasks[t];
    const DCod c = load_cod(a.cods + tk.cod);
    const int k = a.k;
    const int lg = KR == 1 ? (tk.meta & 0xff) : 0;
    const int G = 1 << lg, P = KR == 1 ? WAVE >> lg : WAVE / KR;
    const int slot = KR == 1 ? lane >> lg : lane / KR, g = KR == 1 ? lane & (G - 1) : 0;
    const int rl = KR == 1 ? 0 : lane % KR;
    const int lanes_per_slice = KR == 1 ? 1 : min(KR, k); // tally count of one slice
    for (int base = tk.i0b; base < tk.i0e; base += P) {
        const int i0 = min(base + slot, tk.i0e - 1);
        const bool active = base + slot < tk.i0e;
        const int64_t row = c.row0 + (int64_t)i0 * c.row_step;
        const int64_t op = c.op0 + (int64_t)i0 * c.op_step;
        const int64_t col = c.col0 + (int64_t)i0 * c.sigma0;
        bool counted = false;
        if constexpr (KR == 1) {
            for (int r = 0; r < k; r++) {
                double acc = 0.0;
                for (int i1 = g; i1 < c.nn; i1 += G)
                    acc += a.vals[op + i1] * a.x[(col + (int64_t)i1 * c.sigma1) * k + r];
                for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
                if (active && g == 0) unsafeAtomicAdd(a.y + row * k + r, acc);
            }
            counted = active && g == 0;
        } else {
            for (int r = rl; r < k; r += KR) {
                double acc = 0.0;
                for (int i1 = 0; i1 < c.nn; i1++) acc += a.vals[op + i1] * a.x[(col + (int64_t)i1 * c.sigma1) * k + r];
                if (active) unsafeAtomicAdd(a.y + row * k + r, acc);
            }
            counted = active && rl < k;
        }
        if constexpr (SOLVE) {
            if (counted) {
                __threadfence();
                const unsigned prev = atomicAdd(a.cnt + row, 1u);
                if (prev + 1 == (unsigned)(a.need[row] * lanes_per_slice)) {
                    __threadfence();
                    const double d = a.vals[a.rp[row + 1] - 1];
                    for (int r = 0; r < k; r++)
                        a.xs[row * k + r] = (a.b[row * k + r] - cload(a.y + row * k + r)) / d;
                }
            }
        }
    }
}

// Before the slices: SpMV zeroes y; the solve zeroes the accumulators and tallies and solves
// the rows that have no ops (x = b / diagonal).
template <bool SOLVE> __global__ __launch_bounds__(256) void k_slices_init(SliceArgs a) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= a.n) return;
    const int k = a.k;
    for (int r = 0; r < k; r++) a.y[row * k + r] = 0.0;
    if constexpr (SOLVE) {
        a.cnt[row] = 0;
        if (a.need[row] == 0) {
            const double d = a.vals[a.rp[row + 1] - 1];
            for (int r = 0; r < k; r++) a.xs[row * k + r] = a.b[row * k + r] / d;
        }
    }
}

int g_solve_blocks = 0; // blocks of the dataflow solve the whole device keeps resident at once
int g_num_cu = 0;

int solve_grid(int ntasks, int want) {
    int cap = g_solve_blocks > 0 ? g_solve_blocks : 1024;
    if (want > 0 && want < cap) cap = want;
    const int need = (ntasks + WPB - 1) / WPB;
    return need < cap ? (need > 0 ? need : 1) : cap;
}

} // namespace

int kt_for(int k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : 8; }

hipError_t init_device_info() {
    if (g_solve_blocks > 0) return hipSuccess;
    int dev = 0, ncu = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_solve_df<8, true, false>, WAVE * WPB, 0);
    if (e != hipSuccess) return e;
    g_num_cu = ncu > 0 ? ncu : 1;
    g_solve_blocks = (nb > 0 ? nb : 1) * g_num_cu;
    return hipSuccess;
}

int kr_for(int k) { return k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : 32; }

hipError_t launch_spmv(const SpmvArgs &a, bool vperm, hipStream_t s) {
    const int nb = (a.ntasks + WPB - 1) / WPB;
    if (nb == 0) return hipSuccess;
    const dim3 grid(nb), block(WAVE * WPB);
    if (a.k == 1) {
        if (vperm) hipLaunchKernelGGL(k_spmv1<true>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(k_spmv1<false>, grid, block, 0, s, a);
        return hipGetLastError();
    }
    // vector right-hand sides when k allows and x, y are 16-byte aligned
    const bool al = ((reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.y)) & 15) == 0;
#define DDF_SPMVNV(KR, RV, KW)                                                                      \
    {                                                                                               \
        if (vperm) hipLaunchKernelGGL((k_spmvN<KR, RV, KW, true>), grid, block, 0, s, a);         \
        else hipLaunchKernelGGL((k_spmvN<KR, RV, KW, false>), grid, block, 0, s, a);               \
        return hipGetLastError();                                                                   \
    }
    if (al && a.k == 2) DDF_SPMVNV(1, 2, 2)
    if (al && a.k == 4) DDF_SPMVNV(1, 4, 4)
    if (al && a.k == 8) DDF_SPMVNV(2, 4, 8)
    if (al && a.k == 16) DDF_SPMVNV(4, 4, 16)
    if (al && a.k == 32) DDF_SPMVNV(8, 4, 32)
#undef DDF_SPMVNV
#define DDF_SPMVN(KR)                                                                               \
    if (vperm) hipLaunchKernelGGL((k_spmvN<KR, 1, KR, true>), grid, block, 0, s, a);             \
    else hipLaunchKernelGGL((k_spmvN<KR, 1, KR, false>), grid, block, 0, s, a);                   \
    break;
    switch (kr_for(a.k)) {
    case 2: DDF_SPMVN(2)
    case 4: DDF_SPMVN(4)
    case 8: DDF_SPMVN(8)
    case 16: DDF_SPMVN(16)
    default: DDF_SPMVN(32)
    }
#undef DDF_SPMVN
    return hipGetLastError();
}

hipError_t launch_reset(unsigned *ctr, int64_t n, hipStream_t s) {
    int64_t nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_reset, dim3((unsigned)nb), dim3(256), 0, s, ctr, n);
    return hipGetLastError();
}

template <int NGS, int LG, bool PIN> static void launch_thin(const ThinArgs &a, dim3 grid, dim3 block, hipStream_t s) {
    hipLaunchKernelGGL((k_solve_thin<1, NGS, LG, PIN>), grid, block, 0, s, a);
}

template <int NGS, bool PIN = false> static void launch_thin_lg(const ThinArgs &a, dim3 grid, dim3 block, hipStream_t s) {
    switch (a.lg) {
    case 0: launch_thin<NGS, 0, PIN>(a, grid, block, s); break;
    case 1: launch_thin<NGS, 1, PIN>(a, grid, block, s); break;
    case 2: launch_thin<NGS, 2, PIN>(a, grid, block, s); break;
    case 3: launch_thin<NGS, 3, PIN>(a, grid, block, s); break;
    case 4: launch_thin<NGS, 4, PIN>(a, grid, block, s); break;
    default: launch_thin<NGS, 5, PIN>(a, grid, block, s); break;
    }
}

hipError_t launch_solve_thin(const ThinArgs &a, int ngs, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (a.nlev == 0) return hipSuccess;
    const dim3 sgrid((unsigned)((a.n_rec + 255) / 256)), rgrid((unsigned)((a.n + 255) / 256)), pblock(256);
    hipLaunchKernelGGL(k_thin_stream, sgrid, pblock, 0, s, a);
    const dim3 grid(1 + 8 * (unsigned)a.helpers), block((unsigned)a.block);
    if (ev0) (void)hipEventRecord(ev0, s);
    // a plan with pinned entries has at most two global slots per lane; the two-slot kernel
    // runs it (a slot without a global operand gathers the zero past the solutions)
    if (a.pins) launch_thin_lg<2, true>(a, grid, block, s);
    else if (ngs == 0) launch_thin_lg<0>(a, grid, block, s);
    else if (ngs == 1) launch_thin_lg<1>(a, grid, block, s);
    else if (ngs == 2) launch_thin_lg<2>(a, grid, block, s);
    else if (ngs == 3) launch_thin_lg<3>(a, grid, block, s);
    else launch_thin_lg<THIN_SLOTS>(a, grid, block, s);
    if (ev1) (void)hipEventRecord(ev1, s);
    hipLaunchKernelGGL(k_thin_scatter, rgrid, pblock, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_thin_codes(const ThinArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_thin_codes, dim3((unsigned)((a.n_rec + 64 + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_slices_init(const SliceArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    if (a.need) hipLaunchKernelGGL(k_slices_init<true>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_slices_init<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

template <int KR> static void launch_slices_kr(const SliceArgs &a, dim3 grid, dim3 block, hipStream_t s) {
    if (a.need) hipLaunchKernelGGL((k_slices<true, KR>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_slices<false, KR>), grid, block, 0, s, a);
}

hipError_t launch_slices(const SliceArgs &a, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.ntasks + WPB - 1) / WPB)), block(WAVE * WPB);
    if (a.k <= 1) launch_slices_kr<1>(a, grid, block, s);
    else if (a.k == 2) launch_slices_kr<2>(a, grid, block, s);
    else if (a.k <= 4) launch_slices_kr<4>(a, grid, block, s);
    else launch_slices_kr<8>(a, grid, block, s);
    return hipGetLastError();
}

// Scratch of the no-allocation entry point: a file-scope device array, one copy per GPU, held
// until the process ends.  Host code uses the address hipGetSymbolAddress gives for the
// current device, never the array's name.
static __device__ __align__(256) double scratch[NOALLOC_CTR_WORDS / 2 + NOALLOC_VALUES];

hipError_t noalloc_scratch(double **ptr) {
    constexpr int MAXDEV = 64;
    static double *addr[MAXDEV] = {nullptr};
    static std::mutex mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

int num_cu() { return g_num_cu > 0 ? g_num_cu : 256; }
int resident_solve_blocks() { return g_solve_blocks > 0 ? g_solve_blocks : 1024; }

// One level's tasks per launch (the launch boundaries order the levels): plain loads and
// stores, no tickets, no waits.  SINGLE (single-matrix calls): four ops' column reads ahead
// of their loads (27-point Laplacian on 170^3: 3% faster; batches of small matrices: 5%
// slower), and the adjoint's values already in U's order.
template <int KT, bool ADJ, bool SINGLE>
__global__ __launch_bounds__(WAVE *WPB) void k_solve_range(SolveArgs a) {
    const int lane = threadIdx.x % WAVE;
    const int t = xcd_block(blockIdx.x, gridDim.x, 1) * WPB + threadIdx.x / WAVE;
    if (t >= a.ntasks) return;
    solve_task<KT, ADJ, false, SINGLE>(a, t, lane);
}

// dst[i] = src[idx[i]], XCD-contiguous ranges (nearby i often share source lines)
__global__ __launch_bounds__(256) void k_gather(double *__restrict__ dst, const double *__restrict__ src,
                                                const int32_t *__restrict__ idx, int64_t n) {
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x, 1) * 256 + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

hipError_t launch_gather(double *dst, const double *src, const int32_t *idx, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, idx, n);
    return hipGetLastError();
}

template <bool SINGLE> static void launch_range(const SolveArgs &a, bool adj, int kt, dim3 grid, dim3 block, hipStream_t s) {
    switch (kt * 2 + (adj ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_solve_range<1, false, SINGLE>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_solve_range<1, true, SINGLE>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_solve_range<2, false, SINGLE>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_solve_range<2, true, SINGLE>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_solve_range<4, false, SINGLE>), grid, block, 0, s, a); break;
    case 9: hipLaunchKernelGGL((k_solve_range<4, true, SINGLE>), grid, block, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_solve_range<8, false, SINGLE>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_solve_range<8, true, SINGLE>), grid, block, 0, s, a); break;
    }
}

hipError_t launch_solve_range(const SolveArgs &a, bool adj, int kt, hipStream_t s) {
    if (a.ntasks == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.ntasks + WPB - 1) / WPB)), block(WAVE * WPB);
    if (a.k_override > 0) launch_range<true>(a, adj, kt, grid, block, s);
    else launch_range<false>(a, adj, kt, grid, block, s);
    return hipGetLastError();
}

// Lanes per row of the dataflow solve for k right-hand sides (a lane per right-hand side, at
// most 8: a pass covers 64, 32, 16 or 8 rows; more right-hand sides loop 8 at a time).  One row
// group per pass for k = 8: rows that wait for different dependences do not share a pass.
int df_lanes(int k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : 8; }

hipError_t launch_fill_u64(void *p, int64_t n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)nb), dim3(256), 0, s, (unsigned long long *)p, n, v);
    return hipGetLastError();
}

// Clears the dataflow solve's ticket, check-in count and mode (not the error flag, which
// ddf_plan_sync_status reads and clears).
__global__ void k_df_reset(unsigned *ctr) {
    const int i = threadIdx.x;
    if (i < CTR_STRIDE) ctr[i] = 0u;
    else if (i < 3 * CTR_STRIDE) ctr[CTR_STRIDE + i] = 0u;
}

hipError_t launch_df_reset(unsigned *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_df_reset, dim3(1), dim3(3 * CTR_STRIDE), 0, s, ctr);
    return hipGetLastError();
}

// The output block [fill, fill + nfill) marked unsolved, then one persistent launch: a.npass
// passes of kr lanes per row, `blocks` 256-thread blocks (0: every block the device keeps
// resident at once).  vperm: the values through perm.
hipError_t launch_solve_df(const SolveArgs &a, bool adj, bool vperm, int kr, int blocks, double *fill, int64_t nfill,
                           hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (a.npass <= 0) return hipSuccess;
    hipError_t e = launch_fill_u64(fill, nfill, DF_SENT_BITS, s);
    if (e != hipSuccess) return e;
    const int nb = solve_grid(a.npass, blocks);
    if (ev0) (void)hipEventRecord(ev0, s);
#define DDF_DF(KR, A, S) hipLaunchKernelGGL((k_solve_df<KR, A, S>), dim3(nb), dim3(WAVE * WPB), 0, s, a)
#define DDF_DF_KR(A, S)                                                                             \
    switch (kr) {                                                                                   \
    case 1: DDF_DF(1, A, S); break;                                                                 \
    case 2: DDF_DF(2, A, S); break;                                                                 \
    case 4: DDF_DF(4, A, S); break;                                                                 \
    default: DDF_DF(8, A, S); break;                                                                \
    }
    if (adj && vperm) DDF_DF_KR(true, true) else if (adj) DDF_DF_KR(true, false) else DDF_DF_KR(false, false)
#undef DDF_DF_KR
#undef DDF_DF
    e = hipGetLastError();
    if (ev1) (void)hipEventRecord(ev1, s);
    return e;
}

static int lg_for(double avg, int ops_per_lane) {
    int lg = 0;
    while (lg < 6 && (double)(1 << lg) * ops_per_lane < avg) lg++;
    return lg;
}

template <int KT, bool VEC, bool EXACT> static void launch_gv_kt(const GvArgs &a, hipStream_t s) {
    if (a.n_chunks > 0) {
        const dim3 cg((unsigned)((a.n_chunks + WPB - 1) / WPB)), cb(WAVE * WPB);
        hipLaunchKernelGGL((k_gv_chunks<KT, VEC, EXACT>), cg, cb, 0, s, a);
    }
    const int R = WAVE >> a.lg;
    if (a.n <= 0) return;
    const dim3 grid((unsigned)((a.n + (int64_t)R * WPB - 1) / ((int64_t)R * WPB))), block(WAVE * WPB);
    hipLaunchKernelGGL((k_gv_csr<KT, VEC, EXACT>), grid, block, 0, s, a);
}

template <int KT> static void launch_gv_vec(const GvArgs &a, bool vec, hipStream_t s) {
    if (a.k == KT) {
        if (vec) launch_gv_kt<KT, true, true>(a, s);
        else launch_gv_kt<KT, false, true>(a, s);
    } else {
        if (vec) launch_gv_kt<KT, true, false>(a, s);
        else launch_gv_kt<KT, false, false>(a, s);
    }
}

hipError_t launch_gv(GvArgs a, double avg_short_row, hipStream_t s) {
    // about two entries a lane: each lane loads its row of g once for both (one entry a lane:
    // 2.59 ms for the SpMV adjoint of the 27-point Laplacian on 170^3 instead of 2.43)
    a.lg = lg_for(avg_short_row, 2);
    if (a.lg > 5) a.lg = 5;
    // 16-byte loads of x rows when every row starts 16-byte aligned
    const bool vec = a.k % 2 == 0 && ((reinterpret_cast<uintptr_t>(a.g) | reinterpret_cast<uintptr_t>(a.x)) & 15) == 0;
    if (a.k <= 1) launch_gv_kt<1, false, true>(a, s);
    else if (a.k <= 2) launch_gv_vec<2>(a, vec, s);
    else if (a.k <= 4) launch_gv_vec<4>(a, vec, s);
    else if (a.k <= 8) launch_gv_vec<8>(a, vec, s);
    else if (a.k <= 16) launch_gv_vec<16>(a, vec, s);
    else launch_gv_vec<32>(a, vec, s);
    return hipGetLastError();
}

bool gv_plan_fits(int32_t k, const double *g, const double *x) {
    const bool al = ((reinterpret_cast<uintptr_t>(g) | reinterpret_cast<uintptr_t>(x)) & 15) == 0;
    return al && (k == 2 || k == 4 || k == 8 || k == 16 || k == 32);
}

hipError_t launch_gv_plan(const GvPlanArgs &a, hipStream_t s) {
    const int nb = (a.ntasks + WPB - 1) / WPB;
    if (nb == 0) return hipSuccess;
    const dim3 grid(nb), block(WAVE * WPB);
    switch (a.k) {
    case 2: hipLaunchKernelGGL((k_gv_plan<1, 2>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_gv_plan<1, 4>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_gv_plan<2, 4>), grid, block, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_gv_plan<4, 4>), grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_gv_plan<8, 4>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KT> static void launch_gv_batch_kt(const GvBatchArgs &a, hipStream_t s) {
    if (a.n_chunks > 0) {
        const dim3 cg((unsigned)((a.n_chunks + WPB - 1) / WPB)), cb(WAVE * WPB);
        hipLaunchKernelGGL((k_gv_batch_chunks<KT>), cg, cb, 0, s, a);
    }
    const int R = WAVE >> a.lg;
    if (a.n <= 0) return;
    const dim3 grid((unsigned)((a.n + (int64_t)R * WPB - 1) / ((int64_t)R * WPB))), block(WAVE * WPB);
    hipLaunchKernelGGL((k_gv_batch<KT>), grid, block, 0, s, a);
}

hipError_t launch_gv_batch_class(GvBatchArgs a, int kt, double avg_short_row, hipStream_t s) {
    a.lg = lg_for(avg_short_row, 2);
    if (a.lg > 5) a.lg = 5;
    a.aligned = ((reinterpret_cast<uintptr_t>(a.g) | reinterpret_cast<uintptr_t>(a.x)) & 15) == 0;
    switch (kt) {
    case 1: launch_gv_batch_kt<1>(a, s); break;
    case 2: launch_gv_batch_kt<2>(a, s); break;
    case 4: launch_gv_batch_kt<4>(a, s); break;
    case 8: launch_gv_batch_kt<8>(a, s); break;
    case 16: launch_gv_batch_kt<16>(a, s); break;
    default: launch_gv_batch_kt<32>(a, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_plain(PlainKind which, PlainArgs a, double avg_row, int kt, hipStream_t s) {
    a.lg = lg_for(avg_row, 4);
    const int R = WAVE >> a.lg;
    int64_t rows = (which == PLAIN_LEVEL) ? (a.hi - a.lo) : a.n;
    if (rows <= 0) return hipSuccess;
    int64_t nb = (rows + (int64_t)R * WPB - 1) / ((int64_t)R * WPB);
    dim3 grid((unsigned)nb), block(WAVE * WPB);
    switch (which) {
    case PLAIN_SPMV:
        if (kt == 1) hipLaunchKernelGGL(k_csr_spmv<1>, grid, block, 0, s, a);
        else if (kt == 2) hipLaunchKernelGGL(k_csr_spmv<2>, grid, block, 0, s, a);
        else if (kt == 4) hipLaunchKernelGGL(k_csr_spmv<4>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(k_csr_spmv<8>, grid, block, 0, s, a);
        break;
    case PLAIN_LEVEL:
        if (kt == 1) hipLaunchKernelGGL(k_csr_level<1>, grid, block, 0, s, a);
        else if (kt == 2) hipLaunchKernelGGL(k_csr_level<2>, grid, block, 0, s, a);
        else if (kt == 4) hipLaunchKernelGGL(k_csr_level<4>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(k_csr_level<8>, grid, block, 0, s, a);
        break;
    case PLAIN_SPMV_ADJ: hipLaunchKernelGGL(k_csr_spmv_adj_atomic, grid, block, 0, s, a); break;
    case PLAIN_GV: hipLaunchKernelGGL(k_csr_gv, grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

} // namespace ddf
