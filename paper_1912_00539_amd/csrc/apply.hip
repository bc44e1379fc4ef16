// Preconditioner application by block Jacobi sweeps on the triangular factors (Algorithm 5 and
// its backward analogue, Section 4.1), and the BSR matrix-vector product.
//
//   forward  y_i <- r_i - sum_{j<i} L_ij y_j          (unit block diagonal: no inverse)
//   backward z_i <- U_ii^{-1} (y_i - sum_{j>i} U_ij z_j)
//
// Each sweep is one launch over all block rows; a quad of 4 lanes owns rpq<T>() block rows (two in
// FP32, one in FP64), lane r owns component r: it reads row r of each block (contiguous across the
// quad) and element r of the gathered 4-vector, the other three elements coming from the quad by
// DPP broadcast. SYNC sweeps read the previous sweep's vector (ping-pong); ASYNC sweeps update in
// place. From the zero initial guess the first forward sweep is y = r, so it is not launched; the
// last forward sweep also produces the first backward sweep z = Dinv y (its rows are at hand).
// Forward sweeps take the rows in ascending workgroup order; backward sweeps and the SpMV may run
// descending, so that a kernel starts on the rows the one before it touched last.
// The chunked sweeps (a forward or backward substitution inside each chunk of consecutive rows)
// run a chunk per workgroup level by level, or a chunk per quad row by row; the single-worker
// sweeps run all rows in one quad.
#include <mutex>
#include <type_traits>

#include "kernels.h"

using namespace abilu;
using namespace abilu_dev;
using namespace abilu_k;

namespace {


// Forward sweep over the strictly lower part of the factor layout (lrow/lcol/Lb).
// Each quad owns rpq<T>() rows (ib, ib + 64) and loads two blocks of each per step (clamped, so
// the loads are branch-free); a row with fewer blocks reads index 0 of the part, which exists
// whenever the loop runs, and discards the product.
template <typename T, typename YI, bool EMIT_Z>
__global__ __launch_bounds__(WG) void k_fwd(int n, const int32_t *__restrict__ lrow, const int32_t *__restrict__ lcol,
                                            const T *__restrict__ Lb, const double *__restrict__ rhs, const YI *yin,
                                            T *yout, const T *__restrict__ Dinv, T *__restrict__ zout) {
    fwd_body<T, YI, EMIT_Z>(blockIdx.x, n, lrow, lcol, Lb, rhs, yin, yout, Dinv, zout);
}

// Backward sweep over the strictly upper part (urow/ucol/Ub), then z_i = Dinv_i (y_i - sum).
// OFFDIAG = false: z = Dinv y only. DUAL: also store z (precision T) into zout2. desc: workgroups
// take the rows in descending order.
template <typename T, typename YI, typename ZO, bool OFFDIAG, bool DUAL>
__global__ __launch_bounds__(WG) void k_bwd(int n, const int32_t *__restrict__ urow, const int32_t *__restrict__ ucol,
                                            const T *__restrict__ Ub, const T *__restrict__ Dinv,
                                            const YI *__restrict__ y, const T *zin, ZO *zout, T *zout2, int desc) {
    const int blk = desc ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
    bwd_body<T, YI, ZO, OFFDIAG, DUAL>(blk, n, urow, ucol, Ub, Dinv, y, zin, zout, zout2);
}

// Single-worker sweeps (ABILU_ASYNC_SERIAL): one quad, in place; forward rows ascending,
// backward rows descending (the second row slot of the body is past the end and skipped).
template <typename T>
__global__ __launch_bounds__(64) void k_fwd_serial(int n, const int32_t *__restrict__ lrow,
                                                   const int32_t *__restrict__ lcol, const T *__restrict__ Lb,
                                                   const double *__restrict__ rhs, T *y) {
    for (int i = 0; i < n; ++i) {
        fwd_rows<T, T, false>(i, n, n, lrow, lcol, Lb, rhs, y, y, (const T *)nullptr, (T *)nullptr);
        __threadfence();
    }
}

template <typename T, typename ZO, bool DUAL>
__global__ __launch_bounds__(64) void k_bwd_serial(int n, const int32_t *__restrict__ urow,
                                                   const int32_t *__restrict__ ucol, const T *__restrict__ Ub,
                                                   const T *__restrict__ Dinv, const T *__restrict__ y, T *zin, ZO *zout) {
    for (int i = n - 1; i >= 0; --i) {
        bwd_rows<T, T, ZO, true, DUAL>(i, n, n, urow, ucol, Ub, Dinv, y, zin, zout, zin);
        __threadfence();
    }
}

template <typename T>
__global__ __launch_bounds__(WG) void k_zero2(int64_t len, T *a, T *b) {
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t < len) {
        a[t] = T(0);
        b[t] = T(0);
    }
}

// Chunked sweeps: workgroup c runs chunk c = rows [c0, c0 + R) level by level, one quad per row,
// with a barrier after each level. Forward: y_i = r_i - sum_{j<i} L_ij y_j, where y_j comes from
// this sweep (yn) for rows of the chunk and from the previous sweep (yo) for earlier rows; in the
// first sweep (ZERO_OUT) the earlier rows contribute their initial value 0 and are not read.
template <typename T, bool ZERO_OUT>
__device__ __forceinline__ void fwd_chunk_row(int i, int c0, const int32_t *__restrict__ lrow,
                                              const int32_t *__restrict__ lcol, const T *__restrict__ Lb,
                                              const double *__restrict__ rhs, const T *yo, T *yn) {
    const int r = threadIdx.x & 3;
    const int b0 = lrow[i], b1 = lrow[i + 1];
    T acc = (T)rhs[(int64_t)i * 4 + r];
    for (int e0 = b0; e0 < b1; e0 += 2) {
        int j[2];
        T l[2][4], yv[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = min(e0 + u, b1 - 1);
            j[u] = lcol[e];
            load_row(Lb + (int64_t)e * BB, r, l[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (j[u] >= c0) yv[u] = yn[(int64_t)j[u] * 4 + r];
            else if constexpr (ZERO_OUT) yv[u] = T(0);
            else yv[u] = yo[(int64_t)j[u] * 4 + r];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            T yj[4];
            gather_vec(yv[u], yj);
            const T c = dot4(l[u][0], yj[0], l[u][1], yj[1], l[u][2], yj[2], l[u][3], yj[3]);
            acc -= (e0 + u < b1) ? c : T(0);
        }
    }
    yn[(int64_t)i * 4 + r] = acc;
}

// Backward: z_i = Dinv_i (y_i - sum_{j>i} U_ij z_j), z_j of this sweep (zn) for rows of the chunk
// (j < c1), of the previous sweep (zo) for later rows, 0 in the first sweep (ZERO_OUT).
template <typename T, typename ZN, bool ZERO_OUT>
__device__ __forceinline__ void bwd_chunk_row(int i, int c1, const int32_t *__restrict__ urow,
                                              const int32_t *__restrict__ ucol, const T *__restrict__ Ub,
                                              const T *__restrict__ Dinv, const T *__restrict__ y, const T *zo,
                                              ZN *zn) {
    const int r = threadIdx.x & 3;
    const int b0 = urow[i], b1 = urow[i + 1];
    T acc = y[(int64_t)i * 4 + r];
    for (int e0 = b0; e0 < b1; e0 += 2) {
        int j[2];
        T u4[2][4], zv[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = min(e0 + u, b1 - 1);
            j[u] = ucol[e];
            load_row(Ub + (int64_t)e * BB, r, u4[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (j[u] < c1) zv[u] = (T)zn[(int64_t)j[u] * 4 + r];
            else if constexpr (ZERO_OUT) zv[u] = T(0);
            else zv[u] = zo[(int64_t)j[u] * 4 + r];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            T zj[4];
            gather_vec(zv[u], zj);
            const T c = dot4(u4[u][0], zj[0], u4[u][1], zj[1], u4[u][2], zj[2], u4[u][3], zj[3]);
            acc -= (e0 + u < b1) ? c : T(0);
        }
    }
    T dr[4], a[4];
    load_row(Dinv + (int64_t)i * BB, r, dr);
    gather_vec(acc, a);
    zn[(int64_t)i * 4 + r] = (ZN)dot4(dr[0], a[0], dr[1], a[1], dr[2], a[2], dr[3], a[3]);
}

template <typename T, bool ZERO_OUT>
__global__ __launch_bounds__(WG) void k_fwd_chunk(int n, int R, const int32_t *__restrict__ order,
                                                  const int32_t *__restrict__ lvptr,
                                                  const int32_t *__restrict__ lvstart,
                                                  const int32_t *__restrict__ lrow, const int32_t *__restrict__ lcol,
                                                  const T *__restrict__ Lb, const double *__restrict__ rhs,
                                                  const T *yo, T *yn) {
    const int c = blockIdx.x, c0 = c * R;
    const int b = lvptr[c], nl = lvptr[c + 1] - b - 1;
    const int quad = threadIdx.x >> 2;
    for (int l = 0; l < nl; ++l) {
        const int p1 = lvstart[b + l + 1];
        for (int q = lvstart[b + l] + quad; q < p1; q += ROWS_PER_WG)
            fwd_chunk_row<T, ZERO_OUT>(order[q], c0, lrow, lcol, Lb, rhs, yo, yn);
        __syncthreads();
    }
}

template <typename T, typename ZN, bool ZERO_OUT>
__global__ __launch_bounds__(WG) void k_bwd_chunk(int n, int R, const int32_t *__restrict__ order,
                                                  const int32_t *__restrict__ lvptr,
                                                  const int32_t *__restrict__ lvstart,
                                                  const int32_t *__restrict__ urow, const int32_t *__restrict__ ucol,
                                                  const T *__restrict__ Ub, const T *__restrict__ Dinv,
                                                  const T *__restrict__ y, const T *zo, ZN *zn) {
    const int c = blockIdx.x, c1 = min(n, c * R + R);
    const int b = lvptr[c], nl = lvptr[c + 1] - b - 1;
    const int quad = threadIdx.x >> 2;
    for (int l = 0; l < nl; ++l) {
        const int p1 = lvstart[b + l + 1];
        for (int q = lvstart[b + l] + quad; q < p1; q += ROWS_PER_WG)
            bwd_chunk_row<T, ZN, ZERO_OUT>(order[q], c1, urow, ucol, Ub, Dinv, y, zo, zn);
        __syncthreads();
    }
}

// The same sweeps with one quad per chunk running its rows in order (forward ascending, backward
// descending); a lane only reads chunk values it stored itself, and takes the element of the row
// computed just before from a register. Each row's operands are located by its record (read one
// row ahead) and fetched together; rows with more than REC_CAP blocks in the part take the general
// row code. The arithmetic and its order are those of fwd_chunk_row / bwd_chunk_row.
template <typename T, bool ZERO_OUT>
__global__ __launch_bounds__(WG) void k_fwd_chunk_rows(int n, int R, int nch, const int32_t *__restrict__ rec,
                                                       const int32_t *__restrict__ lrow,
                                                       const int32_t *__restrict__ lcol, const T *__restrict__ Lb,
                                                       const double *__restrict__ rhs, const T *yo, T *yn) {
    const int c = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    if (c >= nch) return;
    const int r = threadIdx.x & 3;
    const int c0 = c * R, m = min(n, c0 + R) - c0;
    T py = T(0);               // y of row i - 1 (this lane's element)
    bool have_prev = false;
    int4 h = rec_quad(rec, R, c, nch, 0, 0), cols = rec_quad(rec, R, c, nch, 0, 1);
    for (int t = 0; t < m; ++t) {
        const int i = c0 + t;
        const int lb = h.y, meta = h.w, nl = meta & 15;
        const int jl[REC_CAP] = {cols.x, cols.y, cols.z, cols.w};
        if (nl > REC_CAP) {
            if (t + 1 < m) {
                h = rec_quad(rec, R, c, nch, t + 1, 0);
                cols = rec_quad(rec, R, c, nch, t + 1, 1);
            }
            fwd_chunk_row<T, ZERO_OUT>(i, c0, lrow, lcol, Lb, rhs, yo, yn);
            have_prev = false;
            continue;
        }
        T acc = (T)rhs[(int64_t)i * 4 + r];
        T l[REC_CAP][4], yv[REC_CAP];
#pragma unroll
        for (int u = 0; u < REC_CAP; ++u)
            if (u < nl) load_row(Lb + (int64_t)(lb + u) * BB, r, l[u]);
#pragma unroll
        for (int u = 0; u < REC_CAP; ++u) {
            if (u < nl) {
                const int src = (meta >> (12 + 2 * u)) & 3;
                if (src == REC_PREV && have_prev) yv[u] = py;
                else if (src != REC_OUT) yv[u] = yn[(int64_t)jl[u] * 4 + r];
                else if constexpr (ZERO_OUT) yv[u] = T(0);
                else yv[u] = yo[(int64_t)jl[u] * 4 + r];
            }
        }
        if (t + 1 < m) {
            h = rec_quad(rec, R, c, nch, t + 1, 0);
            cols = rec_quad(rec, R, c, nch, t + 1, 1);
        }
#pragma unroll
        for (int u = 0; u < REC_CAP; ++u) {
            if (u < nl) {
                T yj[4];
                gather_vec(yv[u], yj);
                acc -= dot4(l[u][0], yj[0], l[u][1], yj[1], l[u][2], yj[2], l[u][3], yj[3]);
            }
        }
        yn[(int64_t)i * 4 + r] = acc;
        py = acc;
        have_prev = true;
    }
}

template <typename T, typename ZN, bool ZERO_OUT>
__global__ __launch_bounds__(WG) void k_bwd_chunk_rows(int n, int R, int nch, const int32_t *__restrict__ rec,
                                                       const int32_t *__restrict__ urow,
                                                       const int32_t *__restrict__ ucol, const T *__restrict__ Ub,
                                                       const T *__restrict__ Dinv, const T *__restrict__ y,
                                                       const T *zo, ZN *zn) {
    const int c = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    if (c >= nch) return;
    const int r = threadIdx.x & 3;
    const int c0 = c * R, c1 = min(n, c0 + R), m = c1 - c0;
    T pz = T(0);               // z of row i + 1 (this lane's element)
    bool have_prev = false;
    int4 h = rec_quad(rec, R, c, nch, m - 1, 0), cols = rec_quad(rec, R, c, nch, m - 1, 5);
    for (int t = m - 1; t >= 0; --t) {
        const int i = c0 + t;
        const int ub = h.z, meta = h.w, nu = (meta >> 4) & 15;
        const int ju[REC_CAP] = {cols.x, cols.y, cols.z, cols.w};
        if (nu > REC_CAP) {
            if (t > 0) {
                h = rec_quad(rec, R, c, nch, t - 1, 0);
                cols = rec_quad(rec, R, c, nch, t - 1, 5);
            }
            bwd_chunk_row<T, ZN, ZERO_OUT>(i, c1, urow, ucol, Ub, Dinv, y, zo, zn);
            have_prev = false;
            continue;
        }
        T acc = y[(int64_t)i * 4 + r];
        T u4[REC_CAP][4], zv[REC_CAP], dr[4];
#pragma unroll
        for (int w = 0; w < REC_CAP; ++w)
            if (w < nu) load_row(Ub + (int64_t)(ub + w) * BB, r, u4[w]);
#pragma unroll
        for (int w = 0; w < REC_CAP; ++w) {
            if (w < nu) {
                const int src = (meta >> (20 + 2 * w)) & 3;
                if (src == REC_PREV && have_prev) zv[w] = pz;
                else if (src != REC_OUT) zv[w] = (T)zn[(int64_t)ju[w] * 4 + r];
                else if constexpr (ZERO_OUT) zv[w] = T(0);
                else zv[w] = zo[(int64_t)ju[w] * 4 + r];
            }
        }
        load_row(Dinv + (int64_t)i * BB, r, dr);
        if (t > 0) {
            h = rec_quad(rec, R, c, nch, t - 1, 0);
            cols = rec_quad(rec, R, c, nch, t - 1, 5);
        }
#pragma unroll
        for (int w = 0; w < REC_CAP; ++w) {
            if (w < nu) {
                T zj[4];
                gather_vec(zv[w], zj);
                acc -= dot4(u4[w][0], zj[0], u4[w][1], zj[1], u4[w][2], zj[2], u4[w][3], zj[3]);
            }
        }
        T a[4];
        gather_vec(acc, a);
        const T z = dot4(dr[0], a[0], dr[1], a[1], dr[2], a[2], dr[3], a[3]);
        zn[(int64_t)i * 4 + r] = (ZN)z;
        pz = z;
        have_prev = true;
    }
}

// Chunks of at most SHORT_CHUNK rows whose rows hold at most REC_CAP blocks in the part swept:
// the quad reads all of its chunk's records at once (lane r those of steps r, r + 4, r + 8,
// r + 12, broadcast by DPP when their step comes), fully unrolls the chunk and fetches the
// operands of step s + LA while it computes step s, so LA memory round trips overlap. Operands
// from other rows of the chunk (not the one computed just before) are read when the step is
// computed, after their stores. Same arithmetic, in the same order, as fwd_chunk_row /
// bwd_chunk_row.
constexpr int SHORT_CHUNK = 16;
constexpr int LOOKAHEAD = 2;

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int L>
__device__ __forceinline__ int qbi(int v) { return __builtin_amdgcn_update_dpp(0, v, L * 0x55, 0xF, 0xF, false); }

template <int L>
__device__ __forceinline__ int4 qbi4(int4 v) { return make_int4(qbi<L>(v.x), qbi<L>(v.y), qbi<L>(v.z), qbi<L>(v.w)); }

// records k = 0 (fields 0-3) and k = K1 of the chunk's steps r, r + 4, r + 8, r + 12 (row of step s:
// c0 + s forward, c0 + m - 1 - s backward; steps past the chunk's rows read its last step's record)
template <bool DESC, int K1>
__device__ __forceinline__ void load_chunk_records(const int32_t *__restrict__ rec, int R, int c, int nch, int m, int r,
                                                   int4 (&h)[4], int4 (&x)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int s = min(r + 4 * k, m - 1);
        const int t = DESC ? m - 1 - s : s;
        h[k] = rec_quad(rec, R, c, nch, t, 0);
        x[k] = rec_quad(rec, R, c, nch, t, K1);
    }
}

template <typename T, bool ZERO_OUT>
__global__ __launch_bounds__(WG) void k_fwd_chunk_short(int n, int R, int nch, const int32_t *__restrict__ rec,
                                                        const T *__restrict__ Lb, const double *__restrict__ rhs,
                                                        const T *yo, T *yn) {
    const int c = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    if (c >= nch) return;
    const int r = threadIdx.x & 3;
    const int c0 = c * R, m = min(n, c0 + R) - c0;
    int4 hr[4], cr[4];
    load_chunk_records<false, 1>(rec, R, c, nch, m, r, hr, cr);
    struct Ops {
        int meta, jl[REC_CAP];
        double b;
        T l[REC_CAP][4];
        T yv[REC_CAP];
    } ring[LOOKAHEAD + 1];
    T py = T(0);   // y of the row computed just before (this lane's element)
    auto issue = [&](auto sc) {
        constexpr int S = decltype(sc)::value;
        Ops &o = ring[S % (LOOKAHEAD + 1)];
        const int4 h = qbi4<S % 4>(hr[S / 4]), x = qbi4<S % 4>(cr[S / 4]);
        o.meta = h.w;
        o.jl[0] = x.x; o.jl[1] = x.y; o.jl[2] = x.z; o.jl[3] = x.w;
        if (S >= m) return;
        const int i = c0 + S, nl = o.meta & 15;
        o.b = rhs[(int64_t)i * 4 + r];
#pragma unroll
        for (int u = 0; u < REC_CAP; ++u)
            if (u < nl) load_row(Lb + (int64_t)(h.y + u) * BB, r, o.l[u]);
#pragma unroll
        for (int u = 0; u < REC_CAP; ++u) {
            T v = T(0);
            if (u < nl && ((o.meta >> (12 + 2 * u)) & 3) == REC_OUT && !ZERO_OUT) v = yo[(int64_t)o.jl[u] * 4 + r];
            o.yv[u] = v;
        }
    };
    static_for<0, LOOKAHEAD>(issue);
    static_for<0, SHORT_CHUNK>([&](auto sc) {
        constexpr int S = decltype(sc)::value;
        if constexpr (S + LOOKAHEAD < SHORT_CHUNK) issue(std::integral_constant<int, S + LOOKAHEAD>{});
        if (S < m) {
            const Ops &o = ring[S % (LOOKAHEAD + 1)];
            const int nl = o.meta & 15;
            T acc = (T)o.b;
#pragma unroll
            for (int u = 0; u < REC_CAP; ++u) {
                if (u < nl) {
                    const int src = (o.meta >> (12 + 2 * u)) & 3;
                    T yv = o.yv[u];
                    if (src == REC_PREV) yv = py;
                    else if (src == REC_CHUNK) yv = yn[(int64_t)o.jl[u] * 4 + r];
                    T yj[4];
                    gather_vec(yv, yj);
                    acc -= dot4(o.l[u][0], yj[0], o.l[u][1], yj[1], o.l[u][2], yj[2], o.l[u][3], yj[3]);
                }
            }
            yn[(int64_t)(c0 + S) * 4 + r] = acc;
            py = acc;
        }
    });
}

template <typename T, typename ZN, bool ZERO_OUT>
__global__ __launch_bounds__(WG) void k_bwd_chunk_short(int n, int R, int nch, const int32_t *__restrict__ rec,
                                                        const T *__restrict__ Ub, const T *__restrict__ Dinv,
                                                        const T *__restrict__ y, const T *zo, ZN *zn) {
    const int c = blockIdx.x * ROWS_PER_WG + (threadIdx.x >> 2);
    if (c >= nch) return;
    const int r = threadIdx.x & 3;
    const int c0 = c * R, m = min(n, c0 + R) - c0;
    int4 hr[4], cr[4];
    load_chunk_records<true, 5>(rec, R, c, nch, m, r, hr, cr);
    struct Ops {
        int meta, ju[REC_CAP];
        T yi;
        T u[REC_CAP][4];
        T dr[4];
        T zv[REC_CAP];
    } ring[LOOKAHEAD + 1];
    T pz = T(0);   // z of the row computed just before (this lane's element)
    auto issue = [&](auto sc) {
        constexpr int S = decltype(sc)::value;
        Ops &o = ring[S % (LOOKAHEAD + 1)];
        const int4 h = qbi4<S % 4>(hr[S / 4]), x = qbi4<S % 4>(cr[S / 4]);
        o.meta = h.w;
        o.ju[0] = x.x; o.ju[1] = x.y; o.ju[2] = x.z; o.ju[3] = x.w;
        if (S >= m) return;
        const int i = c0 + m - 1 - S, nu = (o.meta >> 4) & 15;
        o.yi = y[(int64_t)i * 4 + r];
#pragma unroll
        for (int w = 0; w < REC_CAP; ++w)
            if (w < nu) load_row(Ub + (int64_t)(h.z + w) * BB, r, o.u[w]);
        load_row(Dinv + (int64_t)i * BB, r, o.dr);
#pragma unroll
        for (int w = 0; w < REC_CAP; ++w) {
            T v = T(0);
            if (w < nu && ((o.meta >> (20 + 2 * w)) & 3) == REC_OUT && !ZERO_OUT) v = zo[(int64_t)o.ju[w] * 4 + r];
            o.zv[w] = v;
        }
    };
    static_for<0, LOOKAHEAD>(issue);
    static_for<0, SHORT_CHUNK>([&](auto sc) {
        constexpr int S = decltype(sc)::value;
        if constexpr (S + LOOKAHEAD < SHORT_CHUNK) issue(std::integral_constant<int, S + LOOKAHEAD>{});
        if (S < m) {
            const Ops &o = ring[S % (LOOKAHEAD + 1)];
            const int i = c0 + m - 1 - S, nu = (o.meta >> 4) & 15;
            T acc = o.yi;
#pragma unroll
            for (int w = 0; w < REC_CAP; ++w) {
                if (w < nu) {
                    const int src = (o.meta >> (20 + 2 * w)) & 3;
                    T zv = o.zv[w];
                    if (src == REC_PREV) zv = pz;
                    else if (src == REC_CHUNK) zv = (T)zn[(int64_t)o.ju[w] * 4 + r];
                    T zj[4];
                    gather_vec(zv, zj);
                    acc -= dot4(o.u[w][0], zj[0], o.u[w][1], zj[1], o.u[w][2], zj[2], o.u[w][3], zj[3]);
                }
            }
            T a[4];
            gather_vec(acc, a);
            const T z = dot4(o.dr[0], a[0], o.dr[1], a[1], o.dr[2], a[2], o.dr[3], a[3]);
            zn[(int64_t)i * 4 + r] = (ZN)z;
            pz = z;
        }
    });
}

// y = A x  (RESID: y = b - A x), double precision, CSR; eight lanes per block row, four blocks
// loaded per step (clamped: rows always hold at least their diagonal block); desc: workgroups
// take the rows in descending order
template <bool RESID>
__global__ __launch_bounds__(WG) void k_spmv(int n, const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ colidx, const double *__restrict__ A,
                                             const double *__restrict__ x, double *__restrict__ y,
                                             const double *__restrict__ b, int desc) {
    const int blk = desc ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
    spmv_body<RESID>(blk, n, rowptr, colidx, A, x, y, b);
}

template <typename T>
const char *tname();
template <>
const char *tname<float>() { return "f32"; }
template <>
const char *tname<double>() { return "f64"; }

template <typename T>
abilu_status apply_t(const abilu_pattern *p, const T *LU, const T *Dinv, const double *r, double *z, int nsw,
                     abilu_mode mode, char *work, const Workspace &W, hipStream_t s) {
    const int n = p->n;
    const int grid = div_up(n, rows_per_wg2<T>());
    const T *Lb = LU;                                              // strictly lower part
    const T *Ub = LU + ((int64_t)p->nnzb_lower + n) * BB;          // strictly upper part
    const int32_t *lrow = p->lrow, *lcol = p->lcol, *urow = p->urow, *ucol = p->ucol;
    T *ya = (T *)(work + W.ya), *yb = (T *)(work + W.yb);
    T *za = (T *)(work + W.za), *zb = (T *)(work + W.zb);
    char name[64];
    auto NAME = [&](const char *base) {
        const char *mn = mode == ABILU_SYNC ? "sync"
                         : mode == ABILU_ASYNC ? "async"
                         : mode == ABILU_ASYNC_SERIAL ? "serial"
                         : mode == ABILU_CHUNK_SYNC ? "chunk_sync" : "chunk_async";
        snprintf(name, sizeof name, "%s_%s_%s", base, tname<T>(), mn);
        return name;
    };
    const Sizes zz = sizes(p);
    const double sF = sizeof(T);
#define LAUNCHED() \
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE

    // From the zero initial guess, sweep 1 forward is y = r and sweep 1 backward is z = Dinv y:
    // they are not launched (the first forward sweep reads r, the last forward sweep also emits
    // z = Dinv y). In ASYNC mode this is the admissible schedule in which no read of sweep 1 sees
    // a value written in the same sweep; sweeps 2..nsw then update y and z in place. SYNC sweeps
    // read the previous sweep's vector (ping-pong ya/yb, za/zb).
    if (mode == ABILU_ASYNC_SERIAL) {
        // zero initial guesses, cleared by a kernel (no memset node if the caller captures a graph)
        const int64_t nv = 4 * (int64_t)n;
        k_zero2<T><<<div_up(nv, WG), WG, 0, s>>>(nv, ya, za);
        LAUNCHED();
        for (int q = 1; q <= nsw; ++q) {
            ProfScope ps(NAME("apply_fwd"), s, bytes_fwd(zz, sF, sF, false));
            k_fwd_serial<T><<<1, 4, 0, s>>>(n, lrow, lcol, Lb, r, ya);
            LAUNCHED();
        }
        for (int q = 1; q <= nsw; ++q) {
            const bool last = q == nsw;
            ProfScope ps(NAME(last ? "apply_bwd_last" : "apply_bwd"), s, bytes_bwd(zz, sF, last ? 8 : sF, last));
            if (last)
                k_bwd_serial<T, double, true><<<1, 4, 0, s>>>(n, urow, ucol, Ub, Dinv, ya, za, z);
            else
                k_bwd_serial<T, T, false><<<1, 4, 0, s>>>(n, urow, ucol, Ub, Dinv, ya, za, za);
            LAUNCHED();
        }
        return ABILU_OK;
    }
    if (mode == ABILU_CHUNK_SYNC || mode == ABILU_CHUNK_ASYNC) {
        // Chunked sweeps, every sweep launched (no closed form: the first sweep already substitutes
        // within each chunk). CHUNK_SYNC: ping-pong ya/yb and za/zb; CHUNK_ASYNC: in place on ya
        // and za; the last backward sweep writes z (double) and reads the chunk's rows from it.
        const bool cs = mode == ABILU_CHUNK_SYNC;
        const int nch = p->nchunks, R = p->chunk_rows;
        const double sch[2] = {4.0 * zz.N + 4.0 * (nch + 1) + 4.0 * (double)(p->total_levels[0] + nch),
                               4.0 * zz.N + 4.0 * (nch + 1) + 4.0 * (double)(p->total_levels[1] + nch)};
        const int32_t *const *O = p->order, *const *LP = p->lvptr, *const *LS = p->lvstart;
        const bool by_rows = p->chunk_runner == ABILU_CHUNK_BY_ROWS;
        const int g = by_rows ? div_up(nch, ROWS_PER_WG) : nch;
        // yo == nullptr: first sweep (earlier rows contribute their initial value 0)
        // chunks of at most SHORT_CHUNK rows whose rows all fit a record: the unrolled runner
        const bool short_fwd = by_rows && R <= SHORT_CHUNK && p->rec_max[0] <= REC_CAP;
        const bool short_bwd = by_rows && R <= SHORT_CHUNK && p->rec_max[1] <= REC_CAP;
        auto fwd = [&](const T *yo, T *yn) {
            if (short_fwd) {
                if (!yo) k_fwd_chunk_short<T, true><<<g, WG, 0, s>>>(n, R, nch, p->rec, Lb, r, yo, yn);
                else k_fwd_chunk_short<T, false><<<g, WG, 0, s>>>(n, R, nch, p->rec, Lb, r, yo, yn);
            } else if (by_rows) {
                if (!yo) k_fwd_chunk_rows<T, true><<<g, WG, 0, s>>>(n, R, nch, p->rec, lrow, lcol, Lb, r, yo, yn);
                else k_fwd_chunk_rows<T, false><<<g, WG, 0, s>>>(n, R, nch, p->rec, lrow, lcol, Lb, r, yo, yn);
            } else {
                if (!yo) k_fwd_chunk<T, true><<<g, WG, 0, s>>>(n, R, O[0], LP[0], LS[0], lrow, lcol, Lb, r, yo, yn);
                else k_fwd_chunk<T, false><<<g, WG, 0, s>>>(n, R, O[0], LP[0], LS[0], lrow, lcol, Lb, r, yo, yn);
            }
        };
        auto bwd = [&](const T *y, const T *zo, auto *zn) {
            using ZN = std::remove_pointer_t<decltype(zn)>;
            if (short_bwd) {
                if (!zo) k_bwd_chunk_short<T, ZN, true><<<g, WG, 0, s>>>(n, R, nch, p->rec, Ub, Dinv, y, zo, zn);
                else k_bwd_chunk_short<T, ZN, false><<<g, WG, 0, s>>>(n, R, nch, p->rec, Ub, Dinv, y, zo, zn);
            } else if (by_rows) {
                if (!zo) k_bwd_chunk_rows<T, ZN, true><<<g, WG, 0, s>>>(n, R, nch, p->rec, urow, ucol, Ub, Dinv, y, zo, zn);
                else k_bwd_chunk_rows<T, ZN, false><<<g, WG, 0, s>>>(n, R, nch, p->rec, urow, ucol, Ub, Dinv, y, zo, zn);
            } else {
                if (!zo)
                    k_bwd_chunk<T, ZN, true><<<g, WG, 0, s>>>(n, R, O[1], LP[1], LS[1], urow, ucol, Ub, Dinv, y, zo, zn);
                else
                    k_bwd_chunk<T, ZN, false><<<g, WG, 0, s>>>(n, R, O[1], LP[1], LS[1], urow, ucol, Ub, Dinv, y, zo, zn);
            }
        };
        const T *yo = nullptr;
        T *yn = ya;
        for (int q = 1; q <= nsw; ++q) {
            yn = (!cs || q % 2 == 1) ? ya : yb;
            ProfScope ps(NAME("apply_fwd"), s, bytes_fwd(zz, sF, sF, false) + sch[0]);
            fwd(q == 1 ? nullptr : (cs ? yo : yn), yn);
            LAUNCHED();
            yo = yn;
        }
        const T *yfin = yn;
        const T *zo = nullptr;
        for (int q = 1; q <= nsw; ++q) {
            const bool last = q == nsw;
            ProfScope ps(NAME(last ? "apply_bwd_last" : "apply_bwd"), s, bytes_bwd(zz, sF, last ? 8 : sF, false) + sch[1]);
            if (last) {
                bwd(yfin, zo, z);
            } else {
                T *zc = (!cs || q % 2 == 1) ? za : zb;
                bwd(yfin, q == 1 ? nullptr : (cs ? zo : zc), zc);
                zo = zc;
            }
            LAUNCHED();
        }
        return ABILU_OK;
    }
    const bool sync = mode == ABILU_SYNC;
    if (nsw == 1) {
        ProfScope ps(NAME("apply_diag"), s, 32 * zz.N + 16 * sF * zz.N + 32 * zz.N);
        k_bwd<T, double, double, false, false><<<grid, WG, 0, s>>>(n, urow, ucol, Ub, Dinv, r, (const T *)nullptr, z,
                                                                   (T *)nullptr, 0);
        LAUNCHED();
        return ABILU_OK;
    }
    const T *yprev = nullptr;   // nullptr: sweep 1, i.e. r itself
    T *ycur = nullptr;
    for (int q = 2; q <= nsw; ++q) {
        ycur = (!sync || q % 2 == 0) ? ya : yb;
        const bool last = (q == nsw);
        ProfScope ps(NAME(last ? "apply_fwd_emitz" : "apply_fwd"), s, bytes_fwd(zz, sF, q == 2 ? 8 : sF, last));
        if (q == 2) {
            if (last)
                k_fwd<T, double, true><<<grid, WG, 0, s>>>(n, lrow, lcol, Lb, r, r, ycur, Dinv, za);
            else
                k_fwd<T, double, false><<<grid, WG, 0, s>>>(n, lrow, lcol, Lb, r, r, ycur, Dinv, (T *)nullptr);
        } else {
            if (last)
                k_fwd<T, T, true><<<grid, WG, 0, s>>>(n, lrow, lcol, Lb, r, yprev, ycur, Dinv, za);
            else
                k_fwd<T, T, false><<<grid, WG, 0, s>>>(n, lrow, lcol, Lb, r, yprev, ycur, Dinv, (T *)nullptr);
        }
        LAUNCHED();
        yprev = ycur;
    }
    const T *yfin = ycur;
    // backward sweeps 2..nsw (sweep 1 produced za). Their workgroup order alternates, starting
    // descending after the ascending forward sweeps, so that each sweep starts on the rows the
    // previous kernel touched last (y, z, Dinv and U there are still in the Infinity Cache). A
    // synchronous sweep's result does not depend on the order; an asynchronous one reads values of
    // the same sweep in either order, and descending is the order of back substitution.
    T *zprev = za;
    for (int q = 2; q <= nsw; ++q) {
        const bool last = (q == nsw);
        const int desc = (q % 2 == 0) ? 1 : 0;
        // ASYNC, last sweep descending: an in-place FP32 copy of z lets the rows updated later in
        // this sweep (the lower ones) read this sweep's values. Ascending, those reads go to rows
        // updated later still, so the copy would serve no read and is not written.
        const bool dual = last && !sync && desc;
        ProfScope ps(NAME(last ? "apply_bwd_last" : "apply_bwd"), s, bytes_bwd(zz, sF, last ? 8 : sF, dual));
        if (last) {
            if (!dual)
                k_bwd<T, T, double, true, false><<<grid, WG, 0, s>>>(n, urow, ucol, Ub, Dinv, yfin, zprev, z, (T *)nullptr,
                                                                     desc);
            else
                k_bwd<T, T, double, true, true><<<grid, WG, 0, s>>>(n, urow, ucol, Ub, Dinv, yfin, zprev, z, zprev, desc);
        } else {
            T *zcur = sync ? ((zprev == za) ? zb : za) : za;
            k_bwd<T, T, T, true, false><<<grid, WG, 0, s>>>(n, urow, ucol, Ub, Dinv, yfin, zprev, zcur, (T *)nullptr, desc);
            zprev = zcur;
        }
        LAUNCHED();
    }
    return ABILU_OK;
#undef LAUNCHED
}

}  // namespace

namespace abilu {

abilu_status apply_impl(const abilu_pattern *p, const void *LU, const void *Dinv, abilu_prec prec, const double *r,
                        double *z, int nsweeps, abilu_mode mode, char *work, const Workspace &W, hipStream_t s) {
    if (p->n == 0) return ABILU_OK;
    if (nsweeps == 0) {
        return hip_ok(hipMemcpyAsync(z, r, sizeof(double) * 4 * (size_t)p->n, hipMemcpyDeviceToDevice, s),
                      "apply identity copy")
                   ? ABILU_OK
                   : ABILU_EDEVICE;
    }
    if (prec == ABILU_F32)
        return apply_t<float>(p, (const float *)LU, (const float *)Dinv, r, z, nsweeps, mode, work, W, s);
    return apply_t<double>(p, (const double *)LU, (const double *)Dinv, r, z, nsweeps, mode, work, W, s);
}

bool apply_ends_descending(int nsweeps, abilu_mode mode) {
    // the last backward sweep q = nsweeps >= 2 of the sweep modes runs descending for even q
    return (mode == ABILU_SYNC || mode == ABILU_ASYNC) && nsweeps >= 2 && nsweeps % 2 == 0;
}

abilu_status spmv_impl(const abilu_pattern *p, const double *A, const double *x, double *y, const double *b,
                       bool desc, hipStream_t s) {
    if (p->n == 0) return ABILU_OK;
    const int grid = div_up(p->n, SPMV_ROWS);
    const Sizes z = sizes(p);
    if (b) {
        ProfScope ps("spmv_resid", s, bytes_spmv(z, true));
        k_spmv<true><<<grid, WG, 0, s>>>(p->n, p->rowptr, p->colidx, A, x, y, b, desc ? 1 : 0);
    } else {
        ProfScope ps("spmv", s, bytes_spmv(z, false));
        k_spmv<false><<<grid, WG, 0, s>>>(p->n, p->rowptr, p->colidx, A, x, y, nullptr, desc ? 1 : 0);
    }
    return launch_status();
}

}  // namespace abilu

extern "C" abilu_status abilu_apply(const abilu_pattern *p, const void *d_LU, const void *d_Dinv, abilu_prec prec,
                                    const double *d_r, double *d_z, int32_t nsweeps, abilu_mode mode, void *d_work,
                                    size_t work_bytes, void *stream) {
    if (!p || nsweeps < 0) return ABILU_EINVAL;
    if (prec != ABILU_F32 && prec != ABILU_F64) return ABILU_EINVAL;
    if (!mode_ok(p, mode)) return ABILU_EINVAL;
    if (!d_work) return ABILU_EINVAL;
    const Workspace W = layout(p, prec, 0);
    if (work_bytes < W.total) return ABILU_EINVAL;
    if (p->n == 0) return ABILU_OK;
    if (!d_r || !d_z || d_r == d_z) return ABILU_EINVAL;
    if (nsweeps > 0 && (!d_LU || !d_Dinv)) return ABILU_EINVAL;
    return apply_impl(p, d_LU, d_Dinv, prec, d_r, d_z, nsweeps, mode, (char *)d_work, W, (hipStream_t)stream);
}

// ------------------------------------------------------------------ allocation-free application
// abilu_apply_noalloc keeps the four apply vectors in this file-scope device array instead of a
// caller workspace. In host code `scratch` names a host-side stand-in, not device memory: its device
// address is obtained once per device with hipGetSymbolAddress (with that device current) and only
// that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[ABILU_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (set up on the first call per device).
abilu_status scratch_ptr(int dev, char **out) {
    if (dev < 0 || dev >= MAX_DEVICES) {
        note_error("abilu_apply_noalloc: device index beyond the library's table");
        return ABILU_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)") || !ptr)
            return ABILU_EDEVICE;
        g_scratch[dev] = (char *)ptr;
    }
    *out = g_scratch[dev];
    return ABILU_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

extern "C" abilu_status abilu_apply_noalloc(const abilu_pattern *p, const void *d_LU, const void *d_Dinv,
                                            abilu_prec prec, const double *d_r, double *d_z, int32_t nsweeps,
                                            abilu_mode mode, void *stream) {
    if (!p || nsweeps < 0) return ABILU_EINVAL;
    if (prec != ABILU_F32 && prec != ABILU_F64) return ABILU_EINVAL;
    if (!mode_ok(p, mode)) return ABILU_EINVAL;
    // the apply vectors ya, yb, za, zb: 4N elements of the factor precision each
    const size_t v = align256((size_t)4 * (size_t)p->n * (prec == ABILU_F32 ? 4 : 8));
    Workspace W{};
    W.ya = 0;
    W.yb = v;
    W.za = 2 * v;
    W.zb = 3 * v;
    W.total = 4 * v;
    if (W.total > (size_t)ABILU_NOALLOC_SCRATCH_BYTES) {
        note_error("abilu_apply_noalloc: the pattern's apply vectors exceed ABILU_NOALLOC_SCRATCH_BYTES");
        return ABILU_EINVAL;
    }
    if (p->n == 0) return ABILU_OK;
    if (!d_r || !d_z || d_r == d_z) return ABILU_EINVAL;
    if (nsweeps > 0 && (!d_LU || !d_Dinv)) return ABILU_EINVAL;
    int dev = -1;
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return ABILU_EDEVICE;
    if (dev != p->device) {
        note_error("abilu_apply_noalloc: the pattern belongs to another device");
        return ABILU_EINVAL;
    }
    char *work = nullptr;
    const abilu_status st = scratch_ptr(dev, &work);
    if (st != ABILU_OK) return st;
    return apply_impl(p, d_LU, d_Dinv, prec, d_r, d_z, nsweeps, mode, work, W, (hipStream_t)stream);
}

extern "C" abilu_status abilu_spmv(const abilu_pattern *p, const double *d_A, const double *d_x, double *d_y,
                                   void *stream) {
    if (!p) return ABILU_EINVAL;
    if (p->n == 0) return ABILU_OK;
    if (!d_A || !d_x || !d_y || d_x == d_y) return ABILU_EINVAL;
    return spmv_impl(p, d_A, d_x, d_y, nullptr, false, (hipStream_t)stream);
}
