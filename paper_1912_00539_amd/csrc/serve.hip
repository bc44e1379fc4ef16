// Continuous batching of independent FGMRES solves (the serving form of the method).
//
// Every admitted request holds one block of the caller's pool with its whole state: the BSR
// system, the factor, the FGMRES workspace and its pattern arrays. A device table of slot
// descriptors points into those blocks. Each tick groups the admitted requests by the step they
// are at (factor + initial residual, Arnoldi step k, end of a restart cycle) and runs each
// kernel of that step once for the whole group: a per-kernel member table lists (slot, first
// tile, k) in ascending tile order, and each workgroup finds its member by binary search and
// runs the same device body as the single-system kernel with its tile index relative to the
// member. Tiles, reductions and stopping decisions are therefore per request, as when it runs
// alone. The host reads one 128-byte status header per slot after each tick to move every
// request to its next step, as fgmres_solve does after each iteration.
//
// Admission runs on a second stream while the device works through the tick: device generation
// of the systems and their pattern analysis, each step one launch for the whole admitted batch
// (member tables over per-request setup descriptors, the bodies of the single-request kernels),
// then the slot descriptors; the compute stream waits on an event before a request's first tick.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "abilu_gen.h"
#include "abilu_serve.h"
#include "kernels.h"
#include "setup_kernels.h"

using namespace abilu;
using namespace abilu_dev;
using namespace abilu_k;

namespace {

constexpr int HDR = 128;        // per-slot status header: flags word at 0, status doubles at 64
constexpr int MAX_SLOTS = 4096;
constexpr int ONE_WG = 64;      // threads per workgroup of the single-lane kernels
constexpr int64_t ADMIT_MIN_CELLS = 1 << 20;   // admission budget per step when few cells are active

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device descriptor of an admitted request.
struct Slot {
    int32_t n, ZL, nb_vec, pad;
    int64_t nv;
    const int32_t *rowptr, *colidx, *diag_pos, *pair_ptr, *pik, *pkj, *sik, *skj, *lrow, *urow, *lcol, *ucol;
    const double *A, *b;
    double *x;
    void *LU, *Dinv, *X1, *D1, *ya, *yb, *za, *zb;
    double *partials, *H, *cs, *sn, *g, *coef, *misc, *red, *V, *Z;
    double *status;
    unsigned *flags;
};

struct Member {
    int32_t slot, tile0, k, pad;
};

// ------------------------------------------------------------------ device side

__device__ __forceinline__ int find_member(const Member *mem, int nmem, int b) {
    int lo = 0, hi = nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mem[mid].tile0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// vector roles, resolved per member
enum { R_VK = 0, R_YA, R_YB, R_ZA, R_ZB, R_ZK, R_VK1, R_V0, R_B, R_X, R_VBASE, R_ZBASE };

__device__ __forceinline__ void *role(const Slot &S, int k, int code) {
    switch (code) {
        case R_VK: return S.V + (int64_t)k * S.nv;
        case R_YA: return S.ya;
        case R_YB: return S.yb;
        case R_ZA: return S.za;
        case R_ZB: return S.zb;
        case R_ZK: return S.Z + (int64_t)k * S.nv;
        case R_VK1: return S.V + (int64_t)(k + 1) * S.nv;
        case R_V0: return S.V;
        case R_B: return (void *)S.b;
        case R_X: return S.x;
        case R_VBASE: return S.V;
        default: return S.Z;
    }
}

#define MEMBER()                                          \
    const int mi_ = find_member(mem, nmem, blockIdx.x);   \
    const Member M = mem[mi_];                            \
    const Slot &S = slots[M.slot];                        \
    const int blk = blockIdx.x - M.tile0

// The same with the launch's tiles taken in descending order when desc is set (as the
// single-system kernels do, so that a kernel starts on the tiles its predecessor touched last).
#define MEMBER_DIR(desc)                                                            \
    const int bid_ = (desc) ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x; \
    const int mi_ = find_member(mem, nmem, bid_);                                   \
    const Member M = mem[mi_];                                                      \
    const Slot &S = slots[M.slot];                                                  \
    const int blk = bid_ - M.tile0

// factor buffers: bit 0 X input is X1, bit 1 D input is D1, bit 2 X output is X1, bit 3 D output is D1
template <typename T>
__device__ __forceinline__ T *fbuf_x(const Slot &S, bool one) { return (T *)(one ? S.X1 : S.LU); }
template <typename T>
__device__ __forceinline__ T *fbuf_d(const Slot &S, bool one) { return (T *)(one ? S.D1 : S.Dinv); }

template <typename T, bool COPY>
__global__ __launch_bounds__(WG) void kb_factor_init(const Slot *slots, const Member *mem, int nmem, int sel) {
    MEMBER_DIR(true);
    factor_init_body<T, double, true, COPY>(blk, S.n, S.ZL, S.rowptr, S.diag_pos, S.lrow, S.urow, S.A,
                                            COPY ? (T *)S.LU : (T *)nullptr, fbuf_d<T>(S, sel & 8), S.flags);
}

template <typename T, bool LA, bool UA, bool DA = false>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(sweep_waves<T>()))) void kb_factor_sweep(const Slot *slots, const Member *mem, int nmem, int sel) {
    MEMBER();
    const T *Xin = (LA && UA) ? (const T *)nullptr : fbuf_x<T>(S, sel & 1);
    factor_sweep_body<T, LA, UA, DA>(blk, S.n, S.ZL, S.rowptr, S.colidx, S.diag_pos, S.lrow, S.urow, S.pair_ptr, S.pik,
                                 S.pkj, S.sik, S.skj, S.A, Xin, UA ? (const T *)nullptr : Xin,
                                 fbuf_d<T>(S, sel & 2), fbuf_x<T>(S, sel & 4), fbuf_d<T>(S, sel & 8), S.flags);
}

template <typename T, typename YI, bool EMIT_Z>
__global__ __launch_bounds__(WG) void kb_fwd(const Slot *slots, const Member *mem, int nmem, int yin, int yout) {
    MEMBER();
    fwd_body<T, YI, EMIT_Z>(blk, S.n, S.lrow, S.lcol, (const T *)S.LU, S.V + (int64_t)M.k * S.nv,
                            (const YI *)role(S, M.k, yin), (T *)role(S, M.k, yout), (const T *)S.Dinv, (T *)S.za);
}

template <typename T, typename YI, typename ZO, bool OFFDIAG, bool DUAL>
__global__ __launch_bounds__(WG) void kb_bwd(const Slot *slots, const Member *mem, int nmem, int y, int zin, int zout,
                                             int desc) {
    MEMBER_DIR(desc);
    const T *Ub = (const T *)S.LU + ((int64_t)S.ZL + S.n) * BB;
    bwd_body<T, YI, ZO, OFFDIAG, DUAL>(blk, S.n, S.urow, S.ucol, Ub, (const T *)S.Dinv, (const YI *)role(S, M.k, y),
                                       (const T *)role(S, M.k, zin), (ZO *)role(S, M.k, zout), (T *)S.za);
}

__global__ __launch_bounds__(WG) void kb_copy(const Slot *slots, const Member *mem, int nmem, int src, int dst) {
    MEMBER();
    const double *s = (const double *)role(S, M.k, src);
    double *d = (double *)role(S, M.k, dst);
    const int64_t base = (int64_t)blk * VEC_TILE + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_E; ++e) {
        const int64_t t = base + (int64_t)e * WG;
        if (t < S.nv) d[t] = s[t];
    }
}

template <bool RESID>
__global__ __launch_bounds__(WG) void kb_spmv(const Slot *slots, const Member *mem, int nmem, int xin, int yout,
                                              int desc) {
    MEMBER_DIR(desc);
    spmv_body<RESID>(blk, S.n, S.rowptr, S.colidx, S.A, (const double *)role(S, M.k, xin),
                     (double *)role(S, M.k, yout), S.b);
}

// q_plus: q = k + q_plus (Arnoldi: k + 1 basis vectors), or q = 0 when q_plus < 0
__global__ __launch_bounds__(WG) void kb_mdot(const Slot *slots, const Member *mem, int nmem, int w, int q_plus,
                                              int use_guard) {
    MEMBER();
    const int q = q_plus < 0 ? 0 : M.k + q_plus;
    mdot_body(blk, S.nv, S.V, S.nv, q, (const double *)role(S, M.k, w), S.partials, S.nb_vec,
              use_guard ? (const int *)(S.misc + MI_GUARD) : nullptr);
}

__global__ __launch_bounds__(WG) void kb_update(const Slot *slots, const Member *mem, int nmem, int base, int q_plus,
                                                double alpha, int w, int with_norm, int use_guard) {
    MEMBER_DIR(true);
    update_body(blk, S.nv, (const double *)role(S, M.k, base), S.nv, M.k + q_plus, S.coef, alpha,
                (double *)role(S, M.k, w), with_norm ? S.partials : nullptr,
                use_guard ? (const int *)(S.misc + MI_GUARD) : nullptr);
}

__global__ __launch_bounds__(WG) void kb_reduce(const Slot *slots, const Member *mem, int nmem, int use_guard) {
    MEMBER();
    reduce_cols_body(blk, S.partials, S.nb_vec, S.red, use_guard ? (const int *)(S.misc + MI_GUARD) : nullptr);
}

// hv = misc[slot]: MI_BETA or MI_HN
__global__ __launch_bounds__(WG) void kb_scale(const Slot *slots, const Member *mem, int nmem, int w, int v, int hslot) {
    MEMBER();
    scale_body(blk, S.nv, (const double *)role(S, M.k, w), (double *)role(S, M.k, v), S.misc + hslot);
}

__global__ __launch_bounds__(WG) void kb_zero(const Slot *slots, const Member *mem, int nmem, int v) {
    MEMBER();
    zero_body(blk, S.nv, (double *)role(S, M.k, v));
}

enum { OP_BETA0 = 0, OP_GS1, OP_GS1_DONE, OP_GS2, OP_GIVENS, OP_SOLVE, OP_BETA_CE };

// single-lane steps on the small dense problem, one lane per member
__global__ void kb_small(const Slot *slots, const Member *mem, int nmem, int op, int m) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nmem) return;
    const Member M = mem[t];
    const Slot &S = slots[M.slot];
    const int k = M.k;
    int *guard = (int *)(S.misc + MI_GUARD);
    switch (op) {
        case OP_BETA0:
            beta_body(0, m, S.red, S.g, S.misc, S.status, ST_NUM);
            beta_body(0, m, S.red, nullptr, S.misc, S.status, ST_BETA);
            break;
        case OP_GS1: gs1_body(0, k, m, S.red, S.H, S.coef, S.misc); break;
        case OP_GS1_DONE: gs1_done_body(0, S.red, S.misc, guard); break;
        case OP_GS2: gs2_body(0, k, m, S.red, S.H, S.coef, guard); break;
        case OP_GIVENS: givens_body(0, k, m, S.red, guard, S.H, S.cs, S.sn, S.g, S.misc, S.status); break;
        case OP_SOLVE: solve_body(0, k, m, S.H, S.g, S.coef); break;
        default: beta_body(0, m, S.red, S.g, S.misc, S.status, ST_BETA); break;
    }
}

// ------------------------------------------------------------------ batched admission kernels
// Generation and pattern analysis of many requests in one launch per step, over per-member
// descriptors and member tables (as the solve kernels), with the bodies of the single-request
// kernels.
struct SetupDesc {
    int32_t n, kind, nx, ny;
    int64_t Z;
    double cfl;
    uint64_t seed;
    int32_t *rowptr, *colidx, *diag_pos, *lrow, *urow, *lcol, *ucol, *pair_ptr, *pik, *pkj, *sik, *skj;
    double *A, *b;
    int64_t *cnt, *ptr64, *tot;   // scratch: 2 x (Z + n + 2) + tiles + 1 int64
    int32_t slot, pad;
};

// scans: row lengths -> rowptr; lower / upper counts -> lrow / urow (totals ZL, ZU); pair counts
// -> pair_ptr (total npairs); adm[4m + 1 + which - 1] receives the totals
enum { SC_ROWPTR = 0, SC_LROW, SC_UROW, SC_PAIR };

// M.slot holds the member's index in the admitted batch (descriptors, staged slots and
// admission words are indexed by it; the table may skip members that failed)
#define SMEMBER()                                         \
    const Member M = mem[find_member(mem, nmem, blockIdx.x)]; \
    const int m_ = M.slot;                                \
    const SetupDesc &D = sd[m_];                          \
    const int blk = blockIdx.x - M.tile0

__device__ __forceinline__ int64_t scan_len(const SetupDesc &D, int which) { return which == SC_PAIR ? D.Z : D.n; }
__device__ __forceinline__ const int64_t *scan_in(const SetupDesc &D, int which) {
    return which == SC_UROW ? D.cnt + (D.n + 1) : D.cnt;
}

__global__ void kbs_gen_rowlen(const SetupDesc *sd, const Member *mem, int nmem) {
    SMEMBER();
    if (D.kind == ABILU_GEN_TRI) abilu_setup::gen_rowlen_body<ABILU_GEN_TRI>(blk, D.nx, D.ny, D.seed, D.n, D.cnt);
    else abilu_setup::gen_rowlen_body<ABILU_GEN_ANISO>(blk, D.nx, D.ny, D.seed, D.n, D.cnt);
}

__global__ __launch_bounds__(WG) void kbs_gen_fill(const SetupDesc *sd, const Member *mem, int nmem) {
    SMEMBER();
    if (D.kind == ABILU_GEN_TRI)
        abilu_setup::gen_fill_body<ABILU_GEN_TRI>(blk, D.nx, D.ny, D.cfl, D.seed, D.n, D.rowptr, D.colidx, D.A, D.b);
    else
        abilu_setup::gen_fill_body<ABILU_GEN_ANISO>(blk, D.nx, D.ny, D.cfl, D.seed, D.n, D.rowptr, D.colidx, D.A, D.b);
}

__global__ __launch_bounds__(abilu_setup::SCAN_T) void kbs_scan_reduce(const SetupDesc *sd, const Member *mem, int nmem,
                                                                      int which) {
    SMEMBER();
    abilu_setup::scan_reduce_body(blk, scan_len(D, which), scan_in(D, which), D.tot);
}

// one workgroup per member
__global__ __launch_bounds__(abilu_setup::SCAN_T) void kbs_scan_totals(const SetupDesc *sd, const Member *mem, int nmem,
                                                                      int which) {
    SMEMBER();
    (void)blk;
    const int nt = div_up(scan_len(D, which) > 0 ? scan_len(D, which) : 1, abilu_setup::SCAN_TILE);
    abilu_setup::scan_totals_body(nt, D.tot, D.tot + nt);
}

__global__ __launch_bounds__(abilu_setup::SCAN_T) void kbs_scan_finish(const SetupDesc *sd, const Member *mem,
                                                                       int nmem, int which, int64_t *adm) {
    SMEMBER();
    const int64_t len = scan_len(D, which);
    const int nt = div_up(len > 0 ? len : 1, abilu_setup::SCAN_TILE);
    int32_t *out32 = which == SC_ROWPTR ? D.rowptr : (which == SC_LROW ? D.lrow : (which == SC_UROW ? D.urow : D.pair_ptr));
    abilu_setup::scan_finish_body(blk, len, scan_in(D, which), D.tot, D.tot + nt, which == SC_PAIR ? D.ptr64 : nullptr,
                                  out32);
    // the member's last workgroup (the one holding index len) records the total for admission
    if (which != SC_ROWPTR && threadIdx.x == 0 && (int64_t)blk == len / abilu_setup::SCAN_TILE)
        adm[4 * m_ + which] = D.tot[nt];
}

__global__ void kbs_pat_rows(const SetupDesc *sd, const Member *mem, int nmem, int64_t *adm) {
    SMEMBER();
    abilu_setup::pat_rows_body(blk, D.n, D.Z, D.rowptr, D.colidx, D.diag_pos, (unsigned *)(adm + 4 * m_));
}

__global__ void kbs_pat_tri_counts(const SetupDesc *sd, const Member *mem, int nmem) {
    SMEMBER();
    abilu_setup::pat_tri_counts_body(blk, D.n, D.rowptr, D.diag_pos, D.cnt, D.cnt + (D.n + 1));
}

__global__ void kbs_pat_count(const SetupDesc *sd, const Member *mem, int nmem) {
    SMEMBER();
    abilu_setup::pat_count_body(blk, D.n, D.rowptr, D.colidx, D.diag_pos, D.cnt);
}

__global__ void kbs_pat_tri_cols(const SetupDesc *sd, const Member *mem, int nmem, const int64_t *adm) {
    SMEMBER();
    abilu_setup::pat_tri_cols_body(blk, D.n, D.rowptr, D.colidx, D.diag_pos, D.lrow, D.urow, D.lcol, D.ucol);
    if (blk == 0 && threadIdx.x == 0) {   // the padding entry after each part
        D.lcol[adm[4 * m_ + SC_LROW]] = 0;
        D.ucol[adm[4 * m_ + SC_UROW]] = 0;
    }
}

__global__ void kbs_pat_fill(const SetupDesc *sd, const Member *mem, int nmem, const int64_t *adm) {
    SMEMBER();
    abilu_setup::pat_fill_body(blk, D.n, (int)adm[4 * m_ + SC_LROW], D.rowptr, D.colidx, D.diag_pos, D.lrow, D.urow,
                               D.ptr64, D.pik, D.pkj, D.sik, D.skj);
}

// Publish member m: its slot descriptor (with ZL from the analysis), a cleared status header and
// cleared scalars. One workgroup per member.
__global__ void kbs_publish(const SetupDesc *sd, const Member *mem, int nmem, const Slot *staged, Slot *slots,
                            char *hdr, const int64_t *adm) {
    SMEMBER();
    (void)blk;
    const int slot = D.slot;
    // copy the staged descriptor word by word (word 0, holding n and ZL, by thread 0, which then
    // sets ZL)
    static_assert(sizeof(Slot) % 8 == 0, "slot descriptor is copied in 8-byte words");
    const uint64_t *src = reinterpret_cast<const uint64_t *>(staged + m_);
    uint64_t *dst = reinterpret_cast<uint64_t *>(slots + slot);
    for (int w = threadIdx.x; w < (int)(sizeof(Slot) / 8); w += blockDim.x) dst[w] = src[w];
    if (threadIdx.x == 0) slots[slot].ZL = (int32_t)adm[4 * m_ + SC_LROW];
    const Slot &v = staged[m_];
    if (threadIdx.x < HDR / 8) ((double *)(hdr + (size_t)slot * HDR))[threadIdx.x] = 0.0;
    if (threadIdx.x < 16) v.misc[threadIdx.x] = 0.0;
}

// ------------------------------------------------------------------ host side

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Pool {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length, disjoint, coalesced
    void init(size_t bytes) {
        size = bytes & ~(size_t)255;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// byte offsets of one request's arrays inside its pool block (NONE: not allocated)
constexpr size_t NONE = ~(size_t)0;
struct ReqLayout {
    size_t rowptr, colidx, diag_pos, pair_ptr, lrow, urow, lcol, ucol, pik, pkj, sik, skj;
    size_t A, b, x, LU, Dinv, X1, D1, ya, yb, za, zb;
    size_t partials, H, cs, sn, g, coef, misc, red, V, Z, scratch;
    size_t total;
    int64_t zcap, pcap;
    int nb_vec;
};

bool config_ok(const abilu_serve_config *c) {
    return c && (c->prec == ABILU_F32 || c->prec == ABILU_F64) && (c->mode == ABILU_SYNC || c->mode == ABILU_ASYNC) &&
           c->factor_sweeps >= 0 && c->apply_sweeps >= 0 && c->restart >= 1 && c->restart <= MAX_RESTART &&
           c->maxit >= 0 && c->rtol >= 0.0 && c->max_active >= 1 && c->max_active <= MAX_SLOTS;
}

ReqLayout req_layout(const abilu_serve_config &c, int32_t n, int64_t Z, size_t gen_scratch) {
    ReqLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    const size_t sF = c.prec == ABILU_F32 ? 4 : 8, nv = 4 * (size_t)n, m = (size_t)c.restart;
    const bool sync = c.mode == ABILU_SYNC;
    // strictly lower/upper parts and update-set lists: at most Z - n entries each (each block
    // of a generated pattern lies in one triangle; its update sets are the diagonal ones)
    L.zcap = Z - n;
    L.pcap = Z - n;
    L.nb_vec = div_up((int64_t)(nv > 0 ? nv : 1), VEC_TILE);
    L.rowptr = take(4 * (size_t)(n + 1));
    L.colidx = take(4 * (size_t)Z);
    L.diag_pos = take(4 * (size_t)(n + 1));
    L.pair_ptr = take(4 * (size_t)(Z + 1));
    L.lrow = take(4 * (size_t)(n + 1));
    L.urow = take(4 * (size_t)(n + 1));
    L.lcol = take(4 * (size_t)(L.zcap + 1));
    L.ucol = take(4 * (size_t)(L.zcap + 1));
    L.pik = take(4 * (size_t)(L.pcap + 1));
    L.pkj = take(4 * (size_t)(L.pcap + 1));
    L.sik = take(4 * (size_t)(L.pcap + 1));
    L.skj = take(4 * (size_t)(L.pcap + 1));
    L.A = take(128 * (size_t)Z);
    L.b = take(8 * nv);
    L.x = take(8 * nv);
    L.LU = take(16 * sF * (size_t)Z);
    L.Dinv = take(16 * sF * (size_t)n);
    L.X1 = (sync && c.factor_sweeps >= 2) ? take(16 * sF * (size_t)Z) : NONE;
    L.D1 = (sync && c.factor_sweeps >= 1) ? take(16 * sF * (size_t)n) : NONE;
    L.ya = take(sF * nv);
    L.za = take(sF * nv);
    L.yb = sync ? take(sF * nv) : NONE;
    L.zb = sync ? take(sF * nv) : NONE;
    L.partials = take(8 * (m + 2) * (size_t)L.nb_vec);
    L.H = take(8 * (m + 1) * m);
    L.cs = take(8 * (m + 2));
    L.sn = take(8 * (m + 2));
    L.g = take(8 * (m + 2));
    L.coef = take(8 * (m + 2));
    L.misc = take(8 * 16);
    L.red = take(8 * (m + 4));
    L.V = take(8 * (m + 1) * nv);
    L.Z = take(8 * m * nv);
    // generation and pattern-analysis scratch reuse the Krylov bases (free until the first tick)
    L.scratch = L.V;
    const size_t need = std::max(pattern_scratch_bytes(n, Z), gen_scratch);
    if (o - L.V < need) o = L.V + align256(need);
    L.total = o;
    return L;
}

enum State { Q_PENDING = 0, Q_READY, Q_FACTOR, Q_ITER, Q_CYCLE_END, Q_DONE };

struct Req {
    abilu_gen_spec spec{};
    double *x_out = nullptr;
    double arrival = 0.0;
    State state = Q_PENDING;
    int slot = -1;
    size_t off = 0;
    ReqLayout L{};
    int32_t n = 0;
    int64_t Z = 0, ZL = 0, ZU = 0, P = 0;   // pattern sizes (after admission)
    int k = 0, iters = 0, restarts = 0, reorth = 0;
    double bnorm = 0, tol = 0, beta = 0, est = 0;
    uint32_t flags = 0;
    abilu_request_result res{};
};

}  // namespace

struct abilu_server {
    abilu_serve_config cfg{};
    char *pool = nullptr;
    Pool alloc;
    int device = 0;
    hipStream_t setup = nullptr;
    Slot *d_slots = nullptr, *h_slots = nullptr;   // h_slots: pinned staging, one per slot
    Member *d_tab = nullptr, *h_tab = nullptr;     // per-tick member tables (pinned staging)
    int tab_cap = 0;
    char *d_hdr = nullptr, *h_hdr = nullptr;       // per-slot status headers
    // batched admission: per-member setup descriptors, staged slot descriptors, member tables
    // and the error/size words read back, device and pinned host copies
    SetupDesc *d_sdesc = nullptr, *h_sdesc = nullptr;
    Slot *d_sslot = nullptr;
    Member *d_stab = nullptr, *h_stab = nullptr;
    int64_t *d_adm = nullptr, *h_adm = nullptr;    // per member: error word, ZL, ZU, npairs
    std::vector<hipEvent_t> ev;                    // per slot: setup finished
    std::vector<Req> reqs;
    std::deque<int64_t> queue;                     // released, not yet admitted (FIFO)
    std::vector<int64_t> slot_req;                 // slot -> request id or -1
    double t0 = 0.0;                               // clock origin
    double stat_bytes = 0.0;                       // algorithmic bytes of the batched launches
    int64_t stat_launches = 0, stat_ticks = 0, stat_admitted = 0, stat_retired = 0;
};

namespace {

// Admission of a batch of requests on the setup stream: every step of generation and pattern
// analysis is one launch for the whole batch, with two stream syncs per batch (error words, then
// the part sizes, are read back). A request whose pattern is invalid or exceeds its reserved
// capacity fails alone.
char *block_ptr(abilu_server *s, const Req &r, size_t o) { return o == NONE ? nullptr : s->pool + r.off + o; }

void release(abilu_server *s, Req &r) {
    if (r.slot >= 0) {
        s->slot_req[r.slot] = -1;
        r.slot = -1;
    }
    s->alloc.release(r.off, r.L.total);
}

void fail_request(abilu_server *s, Req &r, abilu_status st) {
    r.state = Q_DONE;
    r.res.status = st;
    r.res.t_done = now_s() - s->t0;
    release(s, r);
}

enum SetupShape { SS_ROW256 = 0, SS_ROW64, SS_ROW128, SS_SCAN_N, SS_SCAN_Z, SS_FIN_N, SS_FIN_Z, SS_ONE, SS_COUNT };

int setup_tiles(const Req &r, int shape) {
    const int64_t n = r.n, Z = r.Z;
    switch (shape) {
        case SS_ROW256: return div_up(n, 256);
        case SS_ROW64: return div_up(n, ROWS_PER_WG);
        case SS_ROW128: return div_up(n, abilu_setup::PAT_ROWS);
        case SS_SCAN_N: return div_up(n > 0 ? n : 1, abilu_setup::SCAN_TILE);
        case SS_SCAN_Z: return div_up(Z > 0 ? Z : 1, abilu_setup::SCAN_TILE);
        case SS_FIN_N: return div_up(n + 1, abilu_setup::SCAN_TILE);
        case SS_FIN_Z: return div_up(Z + 1, abilu_setup::SCAN_TILE);
        default: return 1;
    }
}

// Member tables of the batch `ids` (member m = position in ids), uploaded to d_stab.
struct SetupTables {
    const Member *d[SS_COUNT];
    int tiles[SS_COUNT];
    int count;
};

abilu_status upload_setup_tables(abilu_server *s, const std::vector<int64_t> &ids, const std::vector<int> &members,
                                 SetupTables &T) {
    int used = 0;
    T.count = (int)members.size();
    for (int sh = 0; sh < SS_COUNT; ++sh) {
        T.d[sh] = s->d_stab + used;
        int tile = 0;
        for (size_t q = 0; q < members.size(); ++q) {
            const Req &r = s->reqs[ids[members[q]]];
            s->h_stab[used + q] = Member{members[q], tile, 0, 0};
            tile += setup_tiles(r, sh);
        }
        T.tiles[sh] = tile;
        used += (int)members.size();
    }
    return hip_ok(hipMemcpyAsync(s->d_stab, s->h_stab, sizeof(Member) * used, hipMemcpyHostToDevice, s->setup),
                  "serve setup tables")
               ? ABILU_OK
               : ABILU_EDEVICE;
}

abilu_status launch_scan(abilu_server *s, const SetupTables &T, int which) {
    const bool z = which == SC_PAIR;
    hipStream_t st = s->setup;
    kbs_scan_reduce<<<T.tiles[z ? SS_SCAN_Z : SS_SCAN_N], abilu_setup::SCAN_T, 0, st>>>(
        s->d_sdesc, T.d[z ? SS_SCAN_Z : SS_SCAN_N], T.count, which);
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    kbs_scan_totals<<<T.tiles[SS_ONE], abilu_setup::SCAN_T, 0, st>>>(s->d_sdesc, T.d[SS_ONE], T.count, which);
    if (launch_status() != ABILU_OK) return ABILU_EDEVICE;
    kbs_scan_finish<<<T.tiles[z ? SS_FIN_Z : SS_FIN_N], abilu_setup::SCAN_T, 0, st>>>(s->d_sdesc, T.d[z ? SS_FIN_Z : SS_FIN_N],
                                                                      T.count, which, s->d_adm);
    return launch_status();
}

void stage_request(abilu_server *s, Req &r, int m) {
    const ReqLayout &L = r.L;
    auto P = [&](size_t o) -> void * { return block_ptr(s, r, o); };
    SetupDesc &D = s->h_sdesc[m];
    D = SetupDesc{};
    D.n = r.n;
    D.kind = r.spec.kind;
    D.nx = r.spec.nx;
    D.ny = r.spec.ny;
    D.Z = r.Z;
    D.cfl = r.spec.cfl;
    D.seed = r.spec.seed;
    D.rowptr = (int32_t *)P(L.rowptr);
    D.colidx = (int32_t *)P(L.colidx);
    D.diag_pos = (int32_t *)P(L.diag_pos);
    D.lrow = (int32_t *)P(L.lrow);
    D.urow = (int32_t *)P(L.urow);
    D.lcol = (int32_t *)P(L.lcol);
    D.ucol = (int32_t *)P(L.ucol);
    D.pair_ptr = (int32_t *)P(L.pair_ptr);
    D.pik = (int32_t *)P(L.pik);
    D.pkj = (int32_t *)P(L.pkj);
    D.sik = (int32_t *)P(L.sik);
    D.skj = (int32_t *)P(L.skj);
    D.A = (double *)P(L.A);
    D.b = (double *)P(L.b);
    const PatScratch S = pat_scratch(P(L.scratch), r.n, r.Z);
    D.cnt = S.cnt;
    D.ptr64 = S.ptr64;
    D.tot = S.tot;
    D.slot = r.slot;
    // the slot descriptor the tick kernels will use (ZL is filled in on the device)
    Slot &d = s->h_slots[m];
    d = Slot{};
    d.n = r.n;
    d.nb_vec = L.nb_vec;
    d.nv = 4 * (int64_t)r.n;
    d.rowptr = D.rowptr;
    d.colidx = D.colidx;
    d.diag_pos = D.diag_pos;
    d.pair_ptr = D.pair_ptr;
    d.pik = D.pik;
    d.pkj = D.pkj;
    d.sik = D.sik;
    d.skj = D.skj;
    d.lrow = D.lrow;
    d.urow = D.urow;
    d.lcol = D.lcol;
    d.ucol = D.ucol;
    d.A = D.A;
    d.b = D.b;
    d.x = (double *)P(L.x);
    d.LU = P(L.LU);
    d.Dinv = P(L.Dinv);
    d.X1 = P(L.X1);
    d.D1 = P(L.D1);
    d.ya = P(L.ya);
    d.yb = P(L.yb);
    d.za = P(L.za);
    d.zb = P(L.zb);
    d.partials = (double *)P(L.partials);
    d.H = (double *)P(L.H);
    d.cs = (double *)P(L.cs);
    d.sn = (double *)P(L.sn);
    d.g = (double *)P(L.g);
    d.coef = (double *)P(L.coef);
    d.misc = (double *)P(L.misc);
    d.red = (double *)P(L.red);
    d.V = (double *)P(L.V);
    d.Z = (double *)P(L.Z);
    d.flags = (unsigned *)(s->d_hdr + (size_t)r.slot * HDR);
    d.status = (double *)(s->d_hdr + (size_t)r.slot * HDR + 64);
}

// Admit queued requests in arrival order while a slot and pool space are free (the head of the
// queue waits for memory; later requests do not overtake it), at most `cell_budget` block rows
// per call beyond the first request: admission then proceeds alongside the ticks instead of
// filling the pool in one burst whose requests would all finish together.
abilu_status admit_queued(abilu_server *s, int64_t cell_budget) {
    std::vector<int64_t> ids;
    int slot = 0;
    int64_t cells = 0;
    while (!s->queue.empty()) {
        if (!ids.empty() && cells + s->reqs[s->queue.front()].n > cell_budget) break;
        while (slot < s->cfg.max_active && s->slot_req[slot] >= 0) ++slot;
        if (slot >= s->cfg.max_active) break;
        Req &r = s->reqs[s->queue.front()];
        size_t off = 0;
        if (!s->alloc.alloc(r.L.total, &off)) break;
        const int64_t id = s->queue.front();
        s->queue.pop_front();
        r.off = off;
        r.slot = slot;
        s->slot_req[slot] = id;
        ids.push_back(id);
        cells += r.n;
    }
    if (ids.empty()) return ABILU_OK;
    hipStream_t st = s->setup;
    const int B = (int)ids.size();
    for (int m = 0; m < B; ++m) stage_request(s, s->reqs[ids[m]], m);
    std::vector<int> members(B);
    for (int m = 0; m < B; ++m) members[m] = m;
    SetupTables T;
#define CKS(x)                                     \
    do {                                           \
        if (!hip_ok((x), #x)) return ABILU_EDEVICE; \
    } while (0)
#define CKL()                                                  \
    do {                                                       \
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE; \
    } while (0)
    CKS(hipMemcpyAsync(s->d_sdesc, s->h_sdesc, sizeof(SetupDesc) * B, hipMemcpyHostToDevice, st));
    CKS(hipMemcpyAsync(s->d_sslot, s->h_slots, sizeof(Slot) * B, hipMemcpyHostToDevice, st));
    CKS(hipMemsetAsync(s->d_adm, 0, sizeof(int64_t) * 4 * B, st));
    if (upload_setup_tables(s, ids, members, T) != ABILU_OK) return ABILU_EDEVICE;
    // pass 1: generation (row lengths, row pointers, blocks and right-hand side) and validation
    kbs_gen_rowlen<<<T.tiles[SS_ROW256], 256, 0, st>>>(s->d_sdesc, T.d[SS_ROW256], T.count);
    CKL();
    if (launch_scan(s, T, SC_ROWPTR) != ABILU_OK) return ABILU_EDEVICE;
    kbs_gen_fill<<<T.tiles[SS_ROW64], WG, 0, st>>>(s->d_sdesc, T.d[SS_ROW64], T.count);
    CKL();
    kbs_pat_rows<<<T.tiles[SS_ROW256], 256, 0, st>>>(s->d_sdesc, T.d[SS_ROW256], T.count, s->d_adm);
    CKL();
    CKS(hipMemcpyAsync(s->h_adm, s->d_adm, sizeof(int64_t) * 4 * B, hipMemcpyDeviceToHost, st));
    CKS(hipStreamSynchronize(st));
    auto keep = [&](auto bad, abilu_status why) -> bool {   // drop failed members, true if any dropped
        std::vector<int> next;
        for (int m : members) {
            Req &r = s->reqs[ids[m]];
            if (bad(m, r)) fail_request(s, r, why);
            else next.push_back(m);
        }
        const bool changed = next.size() != members.size();
        members.swap(next);
        return changed;
    };
    if (keep([&](int m, const Req &) { return *(const unsigned *)(s->h_adm + 4 * m) != 0; }, ABILU_EPATTERN)) {
        if (members.empty()) return ABILU_OK;
        if (upload_setup_tables(s, ids, members, T) != ABILU_OK) return ABILU_EDEVICE;
    }
    // pass 2: lower / upper part offsets and update-set offsets, with their totals
    kbs_pat_tri_counts<<<T.tiles[SS_ROW256], 256, 0, st>>>(s->d_sdesc, T.d[SS_ROW256], T.count);
    CKL();
    if (launch_scan(s, T, SC_LROW) != ABILU_OK || launch_scan(s, T, SC_UROW) != ABILU_OK) return ABILU_EDEVICE;
    kbs_pat_count<<<T.tiles[SS_ROW128], abilu_setup::PAT_ROWS, 0, st>>>(s->d_sdesc, T.d[SS_ROW128], T.count);
    CKL();
    if (launch_scan(s, T, SC_PAIR) != ABILU_OK) return ABILU_EDEVICE;
    CKS(hipMemcpyAsync(s->h_adm, s->d_adm, sizeof(int64_t) * 4 * B, hipMemcpyDeviceToHost, st));
    CKS(hipStreamSynchronize(st));
    if (keep(
            [&](int m, const Req &r) {
                const int64_t *sz = s->h_adm + 4 * m + 1;
                return !pattern_sizes_ok(r.n, r.Z, sz) || sz[0] > r.L.zcap || sz[1] > r.L.zcap || sz[2] > r.L.pcap;
            },
            ABILU_EPATTERN)) {
        if (members.empty()) return ABILU_OK;
        if (upload_setup_tables(s, ids, members, T) != ABILU_OK) return ABILU_EDEVICE;
    }
    // pass 3: part columns, update-set lists, slot descriptors; the compute stream waits on the
    // per-slot events before a request's first tick
    kbs_pat_tri_cols<<<T.tiles[SS_ROW256], 256, 0, st>>>(s->d_sdesc, T.d[SS_ROW256], T.count, s->d_adm);
    CKL();
    kbs_pat_fill<<<T.tiles[SS_ROW128], abilu_setup::PAT_ROWS, 0, st>>>(s->d_sdesc, T.d[SS_ROW128], T.count, s->d_adm);
    CKL();
    kbs_publish<<<T.tiles[SS_ONE], 64, 0, st>>>(s->d_sdesc, T.d[SS_ONE], T.count, s->d_sslot, s->d_slots, s->d_hdr,
                                                 s->d_adm);
    CKL();
    const double t = now_s() - s->t0;
    for (int m : members) {
        Req &r = s->reqs[ids[m]];
        const int64_t *sz = s->h_adm + 4 * m + 1;
        r.ZL = sz[0];
        r.ZU = sz[1];
        r.P = sz[2];
        CKS(hipEventRecord(s->ev[r.slot], st));
        r.state = Q_READY;
        r.res.t_admit = t;
        ++s->stat_admitted;
    }
    // the staging buffers are rewritten by the next admission: let this one finish first
    CKS(hipStreamSynchronize(st));
    return ABILU_OK;
#undef CKS
#undef CKL
}

// ---- per-tick member tables
// SH_APPLY: rows_per_wg2<T>() rows per tile; SH_SPMV: SPMV_ROWS rows per tile
enum Shape { SH_ROW64 = 0, SH_APPLY, SH_VEC, SH_COLSQ, SH_ONE, SH_SPMV, SH_COUNT };

struct Table {
    const Member *d = nullptr;
    int count = 0, tiles = 0;
};

int tiles_of(const Req &r, int shape, State g, abilu_prec prec) {
    switch (shape) {
        case SH_ROW64: return div_up(r.n, ROWS_PER_WG);
        case SH_APPLY: return div_up(r.n, prec == ABILU_F32 ? rows_per_wg2<float>() : rows_per_wg2<double>());
        case SH_VEC: return r.L.nb_vec;
        case SH_SPMV: return div_up(r.n, SPMV_ROWS);
        case SH_COLSQ: return g == Q_ITER ? r.k + 2 : 1;
        default: return 1;
    }
}

struct Group {
    State st;
    std::vector<int64_t> ids;
    Table t[SH_COUNT];
    int pass2 = 0;              // profile slot of the first launch of the second Gram-Schmidt pass
};

// Kernel launches of one group (identical sequence for every member). Every launch is recorded
// with the sum over its members of the single-system kernel's algorithmic bytes.
template <typename T>
abilu_status run_group(abilu_server *s, Group &G, hipStream_t st) {
    const abilu_serve_config &c = s->cfg;
    const Slot *sl = s->d_slots;
    const int m = c.restart;
    const int nsw = c.apply_sweeps, fsw = c.factor_sweeps;
    const bool sync = c.mode == ABILU_SYNC;
    const double sF = sizeof(T);
    // sum of f(sizes, request) over the members
    auto B = [&](auto f) {
        double b = 0;
        for (int64_t id : G.ids) {
            const Req &r = s->reqs[id];
            b += f(Sizes{(double)r.n, (double)r.Z, (double)r.ZL, (double)r.ZU, (double)r.P}, r);
        }
        s->stat_bytes += b;
        ++s->stat_launches;
        return b;
    };
    auto nv8 = [](const Sizes &z) { return 32.0 * z.N; };   // bytes of one FP64 Krylov vector
#define L_(shape) dim3(G.t[shape].tiles), dim3(WG), 0, st
#define A_(shape) sl, G.t[shape].d, G.t[shape].count
#define ONE_() dim3(div_up(G.t[SH_ONE].count, ONE_WG)), dim3(ONE_WG), 0, st
#define CKL()                                                  \
    do {                                                       \
        if (launch_status() != ABILU_OK) return ABILU_EDEVICE; \
    } while (0)
    // dots of w with V_0..V_{q-1} and ||w||^2; q = k + q_plus, or 0 when q_plus < 0
    auto mdot = [&](int w, int q_plus, int guard) -> abilu_status {
        auto qof = [&](const Req &r) { return q_plus < 0 ? 0 : r.k + q_plus; };
        {
            ProfScope ps("serve_mdot", st, B([&](const Sizes &z, const Req &r) { return (qof(r) + 1) * nv8(z); }));
            kb_mdot<<<L_(SH_VEC)>>>(A_(SH_VEC), w, q_plus, guard);
        }
        CKL();
        {
            ProfScope ps("serve_reduce", st,
                         B([&](const Sizes &, const Req &r) { return 8.0 * (qof(r) + 1) * r.L.nb_vec; }));
            if (q_plus < 0)
                kb_reduce<<<L_(SH_ONE)>>>(A_(SH_ONE), guard);
            else
                kb_reduce<<<L_(SH_COLSQ)>>>(A_(SH_COLSQ), guard);
        }
        CKL();
        return ABILU_OK;
    };
    // w += alpha sum_k coef_k base_k over q = k + q_plus vectors (+ ||w||^2 partials)
    auto update = [&](int base, int q_plus, double alpha, int w, int norm, int guard) -> abilu_status {
        {
            ProfScope ps("serve_update", st,
                         B([&](const Sizes &z, const Req &r) { return (r.k + q_plus + 2) * nv8(z); }));
            kb_update<<<L_(SH_VEC)>>>(A_(SH_VEC), base, q_plus, alpha, w, norm, guard);
        }
        CKL();
        if (norm) {
            ProfScope ps("serve_reduce", st, B([&](const Sizes &, const Req &r) { return 8.0 * r.L.nb_vec; }));
            kb_reduce<<<L_(SH_ONE)>>>(A_(SH_ONE), guard);
            CKL();
        }
        return ABILU_OK;
    };
    auto small = [&](int op) -> abilu_status {
        ProfScope ps("serve_small", st, B([](const Sizes &, const Req &) { return 0.0; }));
        kb_small<<<ONE_()>>>(A_(SH_ONE), op, m);
        CKL();
        return ABILU_OK;
    };
    auto scale = [&](int w, int v, int hslot) -> abilu_status {
        ProfScope ps("serve_scale", st, B([&](const Sizes &z, const Req &) { return 2 * nv8(z); }));
        kb_scale<<<L_(SH_VEC)>>>(A_(SH_VEC), w, v, hslot);
        CKL();
        return ABILU_OK;
    };
    auto init = [&](bool copy, int sel) -> abilu_status {
        ProfScope ps("serve_factor_init", st, B([&](const Sizes &z, const Req &) { return bytes_init(z, 8, sF, copy); }));
        if (copy)
            kb_factor_init<T, true><<<L_(SH_ROW64)>>>(A_(SH_ROW64), sel);
        else
            kb_factor_init<T, false><<<L_(SH_ROW64)>>>(A_(SH_ROW64), sel);
        CKL();
        return ABILU_OK;
    };
    auto fwd = [&](const char *name, bool yin_f64, bool emit, int yin, int yout) -> abilu_status {
        ProfScope ps(name, st, B([&](const Sizes &z, const Req &) { return bytes_fwd(z, sF, yin_f64 ? 8 : sF, emit); }));
        if (yin_f64) {
            if (emit) kb_fwd<T, double, true><<<L_(SH_APPLY)>>>(A_(SH_APPLY), yin, yout);
            else kb_fwd<T, double, false><<<L_(SH_APPLY)>>>(A_(SH_APPLY), yin, yout);
        } else {
            if (emit) kb_fwd<T, T, true><<<L_(SH_APPLY)>>>(A_(SH_APPLY), yin, yout);
            else kb_fwd<T, T, false><<<L_(SH_APPLY)>>>(A_(SH_APPLY), yin, yout);
        }
        CKL();
        return ABILU_OK;
    };
    // the Arnoldi SpMV runs opposite to the last backward sweep (descending for even q), the
    // residual SpMV descending
    const bool spmv_desc = !(nsw >= 2 && nsw % 2 == 0);
    auto spmv = [&](bool resid, int xin, int yout) -> abilu_status {
        ProfScope ps(resid ? "serve_spmv_resid" : "serve_spmv", st,
                     B([&](const Sizes &z, const Req &) { return bytes_spmv(z, resid); }));
        if (resid)
            kb_spmv<true><<<L_(SH_SPMV)>>>(A_(SH_SPMV), xin, yout, 1);
        else
            kb_spmv<false><<<L_(SH_SPMV)>>>(A_(SH_SPMV), xin, yout, spmv_desc ? 1 : 0);
        CKL();
        return ABILU_OK;
    };
    abilu_status e;
    if (G.st == Q_FACTOR) {
        if (fsw == 0) {
            if ((e = init(true, 0)) != ABILU_OK) return e;
        } else if (!sync) {
            // the first sweep forms the initial inverses inv(A_jj) itself (no initialisation pass)
            {
                ProfScope ps("serve_factor_sweep_fromA", st,
                             B([&](const Sizes &z, const Req &) { return bytes_sweep_from_a(z, sF, false); }));
                kb_factor_sweep<T, false, true, true><<<L_(SH_ROW64)>>>(A_(SH_ROW64), 0);
            }
            CKL();
            for (int q = 1; q < fsw; ++q) {
                ProfScope ps("serve_factor_sweep", st,
                             B([&](const Sizes &z, const Req &) { return bytes_sweep(z, sF, false, false); }));
                kb_factor_sweep<T, false, false><<<L_(SH_ROW64)>>>(A_(SH_ROW64), 0);
                CKL();
            }
        } else {
            // sweep q writes X1/D1 when (fsw - q) is odd, LU/Dinv when even (the last is LU/Dinv)
            auto one = [&](int q) { return ((fsw - q) % 2) != 0; };
            // the first sweep forms the initial inverses inv(A_jj) itself (no initialisation pass)
            {
                ProfScope ps("serve_factor_sweep_fromA", st,
                             B([&](const Sizes &z, const Req &) { return bytes_sweep_from_a(z, sF, true); }));
                kb_factor_sweep<T, true, true, true>
                    <<<L_(SH_ROW64)>>>(A_(SH_ROW64), (one(0) ? 2 : 0) | (one(1) ? 4 : 0) | (one(1) ? 8 : 0));
            }
            CKL();
            for (int q = 2; q <= fsw; ++q) {
                const int sel = (one(q - 1) ? 3 : 0) | (one(q) ? 12 : 0);
                ProfScope ps("serve_factor_sweep", st,
                             B([&](const Sizes &z, const Req &) { return bytes_sweep(z, sF, false, false); }));
                kb_factor_sweep<T, false, false><<<L_(SH_ROW64)>>>(A_(SH_ROW64), sel);
                CKL();
            }
        }
        // ||b||; zero initial guess: beta = ||b||, V_0 = b / beta
        if ((e = mdot(R_B, -1, 0)) != ABILU_OK) return e;
        if ((e = small(OP_BETA0)) != ABILU_OK) return e;
        {
            ProfScope ps("serve_zero", st, B([&](const Sizes &z, const Req &) { return nv8(z); }));
            kb_zero<<<L_(SH_VEC)>>>(A_(SH_VEC), R_X);
        }
        CKL();
        return scale(R_B, R_V0, MI_BETA);
    }
    if (G.st == Q_ITER) {
        // z_k = M^{-1} v_k
        if (nsw == 0) {
            ProfScope ps("serve_apply_copy", st, B([&](const Sizes &z, const Req &) { return 2 * nv8(z); }));
            kb_copy<<<L_(SH_VEC)>>>(A_(SH_VEC), R_VK, R_ZK);
            CKL();
        } else if (nsw == 1) {
            ProfScope ps("serve_apply_diag", st,
                         B([&](const Sizes &z, const Req &) { return 32 * z.N + 16 * sF * z.N + 32 * z.N; }));
            kb_bwd<T, double, double, false, false><<<L_(SH_APPLY)>>>(A_(SH_APPLY), R_VK, R_ZA, R_ZK, 0);
            CKL();
        } else {
            // sweep 1 forward is y = v_k and sweep 1 backward z = Dinv y (emitted by the last forward
            // sweep); ASYNC sweeps 2.. update in place, SYNC sweeps ping-pong
            int yprev = R_VK, ycur = R_YA;
            for (int q = 2; q <= nsw; ++q) {
                ycur = (!sync || q % 2 == 0) ? R_YA : R_YB;
                const bool last = q == nsw;
                if ((e = fwd(last ? "serve_apply_fwd_emitz" : "serve_apply_fwd", q == 2, last, yprev, ycur)) != ABILU_OK)
                    return e;
                yprev = ycur;
            }
            int zprev = R_ZA;
            for (int q = 2; q <= nsw; ++q) {
                const bool last = q == nsw;
                const bool dual = last && !sync && q % 2 == 0;   // the in-place copy serves only a descending sweep
                ProfScope ps(last ? "serve_apply_bwd_last" : "serve_apply_bwd", st,
                             B([&](const Sizes &z, const Req &) { return bytes_bwd(z, sF, last ? 8 : sF, dual); }));
                if (last) {
                    if (dual)
                        kb_bwd<T, T, double, true, true><<<L_(SH_APPLY)>>>(A_(SH_APPLY), ycur, zprev, R_ZK, q % 2 == 0);
                    else
                        kb_bwd<T, T, double, true, false><<<L_(SH_APPLY)>>>(A_(SH_APPLY), ycur, zprev, R_ZK, q % 2 == 0);
                } else {
                    const int zcur = sync ? ((zprev == R_ZA) ? R_ZB : R_ZA) : R_ZA;
                    kb_bwd<T, T, T, true, false><<<L_(SH_APPLY)>>>(A_(SH_APPLY), ycur, zprev, zcur, q % 2 == 0);
                    zprev = zcur;
                }
                CKL();
            }
        }
        if ((e = spmv(false, R_ZK, R_VK1)) != ABILU_OK) return e;
        // Gram-Schmidt pass 1, then pass 2 only where the device set the guard
        if ((e = mdot(R_VK1, 1, 0)) != ABILU_OK) return e;
        if ((e = small(OP_GS1)) != ABILU_OK) return e;
        if ((e = update(R_VBASE, 1, -1.0, R_VK1, 1, 0)) != ABILU_OK) return e;
        if ((e = small(OP_GS1_DONE)) != ABILU_OK) return e;
        // launches pass2 .. pass2 + 4: mdot, reduce, gs2, update, reduce (bytes corrected after
        // the tick for members whose guard stayed clear)
        G.pass2 = prof_mark();
        if ((e = mdot(R_VK1, 1, 1)) != ABILU_OK) return e;
        if ((e = small(OP_GS2)) != ABILU_OK) return e;
        if ((e = update(R_VBASE, 1, -1.0, R_VK1, 1, 1)) != ABILU_OK) return e;
        if ((e = small(OP_GIVENS)) != ABILU_OK) return e;
        return scale(R_VK1, R_VK1, MI_HN);
    }
    // end of a restart cycle over k Arnoldi steps: x += Z y, true residual, next V_0
    if ((e = small(OP_SOLVE)) != ABILU_OK) return e;
    if ((e = update(R_ZBASE, 0, 1.0, R_X, 0, 0)) != ABILU_OK) return e;
    if ((e = spmv(true, R_X, R_V0)) != ABILU_OK) return e;
    if ((e = mdot(R_V0, -1, 0)) != ABILU_OK) return e;
    if ((e = small(OP_BETA_CE)) != ABILU_OK) return e;
    return scale(R_V0, R_V0, MI_BETA);
#undef L_
#undef A_
#undef ONE_
#undef CKL
}

void finish(abilu_server *s, Req &r, bool converged, bool nonfinite) {
    abilu_request_result &o = r.res;
    const double bn = r.bnorm > 0 ? r.bnorm : 1.0;
    o.n = r.n;
    o.nnzb = r.Z;
    o.iters = r.iters;
    o.restarts = r.restarts;
    o.converged = converged ? 1 : 0;
    o.reorth = r.reorth;
    o.flags = r.flags;
    o.rel_true_residual = r.beta / bn;
    o.footprint_bytes = (int64_t)r.L.total;
    o.status = nonfinite ? ABILU_ENONFINITE
                         : (!converged ? ABILU_WARN_NOCONV : ((r.flags & ABILU_FLAG_MODIFIED) ? ABILU_WARN_MODIFIED : ABILU_OK));
    r.state = Q_DONE;
}

// Move a member to its next step from its status header (the decisions fgmres_solve takes).
void advance(abilu_server *s, Req &r) {
    const abilu_serve_config &c = s->cfg;
    const char *h = s->h_hdr + (size_t)r.slot * HDR;
    const double *stv = (const double *)(h + 64);
    r.flags = *(const uint32_t *)h;
    if (r.state == Q_FACTOR) {
        r.bnorm = stv[ST_NUM];
        r.beta = stv[ST_BETA];
        r.est = r.beta;
        r.tol = c.rtol * (r.bnorm > 0 ? r.bnorm : 1.0);
        const bool nonfinite = !std::isfinite(r.beta) || !std::isfinite(r.bnorm);
        const bool conv = r.beta <= r.tol;
        if (conv || nonfinite || c.maxit == 0 || r.beta == 0.0) {
            finish(s, r, conv, nonfinite);
            return;
        }
        r.state = Q_ITER;
        r.k = 0;
        return;
    }
    if (r.state == Q_ITER) {
        if (stv[ST_GUARD] != 0.0) ++r.reorth;
        ++r.iters;
        ++r.k;
        r.est = stv[ST_EST];
        if (!std::isfinite(r.est) || !std::isfinite(stv[ST_HN])) {
            finish(s, r, false, true);
            return;
        }
        if (r.est <= r.tol || stv[ST_HN] == 0.0 || r.k == c.restart || r.iters >= c.maxit) r.state = Q_CYCLE_END;
        return;
    }
    // cycle end
    ++r.restarts;
    r.beta = stv[ST_BETA];
    const bool nonfinite = !std::isfinite(r.beta);
    const bool conv = r.beta <= r.tol;
    if (conv || nonfinite || r.iters >= c.maxit || r.beta == 0.0) {
        finish(s, r, conv && !nonfinite, nonfinite);
        return;
    }
    r.state = Q_ITER;
    r.k = 0;
}

abilu_status step_impl(abilu_server *s, hipStream_t st) {
    abilu_status e;
    Group groups[3] = {{Q_FACTOR, {}, {}}, {Q_ITER, {}, {}}, {Q_CYCLE_END, {}, {}}};
    for (int q = 0; q < s->cfg.max_active; ++q) {
        const int64_t id = s->slot_req[q];
        if (id < 0) continue;
        Req &r = s->reqs[id];
        if (r.state == Q_READY) {
            if (!hip_ok(hipStreamWaitEvent(st, s->ev[q], 0), "serve wait setup")) return ABILU_EDEVICE;
            r.state = Q_FACTOR;
        }
        if (r.state == Q_FACTOR) groups[0].ids.push_back(id);
        else if (r.state == Q_ITER) groups[1].ids.push_back(id);
        else if (r.state == Q_CYCLE_END) groups[2].ids.push_back(id);
    }
    int used = 0;
    for (Group &G : groups) {
        if (G.ids.empty()) continue;
        for (int sh = 0; sh < SH_COUNT; ++sh) {
            Table &T = G.t[sh];
            T.d = s->d_tab + used;
            T.count = (int)G.ids.size();
            int tile = 0;
            for (size_t q = 0; q < G.ids.size(); ++q) {
                const Req &r = s->reqs[G.ids[q]];
                s->h_tab[used + q] = Member{r.slot, tile, r.k, 0};
                tile += tiles_of(r, sh, G.st, (abilu_prec)s->cfg.prec);
            }
            T.tiles = tile;
            used += T.count;
        }
    }
    int64_t tick_cells = 0;
    for (const Group &G : groups)
        for (int64_t id : G.ids) tick_cells += s->reqs[id].n;
    const int64_t budget = std::max<int64_t>(ADMIT_MIN_CELLS, tick_cells);
    if (used == 0) return admit_queued(s, budget);
    if (!hip_ok(hipMemcpyAsync(s->d_tab, s->h_tab, sizeof(Member) * used, hipMemcpyHostToDevice, st), "serve tables"))
        return ABILU_EDEVICE;
    for (Group &G : groups) {
        if (G.ids.empty()) continue;
        e = s->cfg.prec == ABILU_F32 ? run_group<float>(s, G, st) : run_group<double>(s, G, st);
        if (e != ABILU_OK) return e;
    }
    if (!hip_ok(hipMemcpyAsync(s->h_hdr, s->d_hdr, (size_t)s->cfg.max_active * HDR, hipMemcpyDeviceToHost, st),
                "serve status readback"))
        return ABILU_EDEVICE;
    // admissions run on the setup stream while the device works through the tick
    if ((e = admit_queued(s, budget)) != ABILU_OK) return e;
    if (!hip_ok(hipStreamSynchronize(st), "serve tick sync")) return ABILU_EDEVICE;
    ++s->stat_ticks;
    // the second Gram-Schmidt pass exited at once where the guard stayed clear: remove its bytes
    {
        Group &G = groups[1];
        double dm = 0, dr = 0, du = 0, dr2 = 0;
        for (int64_t id : G.ids) {
            const Req &r = s->reqs[id];
            const double *stv = (const double *)(s->h_hdr + (size_t)r.slot * HDR + 64);
            if (stv[ST_GUARD] != 0.0) continue;
            const double nv8 = 32.0 * r.n, q = r.k + 1;
            dm += (q + 1) * nv8;
            dr += 8.0 * (q + 1) * r.L.nb_vec;
            du += (q + 2) * nv8;
            dr2 += 8.0 * r.L.nb_vec;
        }
        s->stat_bytes -= dm + dr + du + dr2;
        if (!G.ids.empty()) {
            prof_add_bytes(G.pass2, -dm);
            prof_add_bytes(G.pass2 + 1, -dr);
            prof_add_bytes(G.pass2 + 3, -du);
            prof_add_bytes(G.pass2 + 4, -dr2);
        }
    }
    // advance, retire finished requests (copy x out first)
    bool copied = false;
    std::vector<int64_t> done;
    for (Group &G : groups)
        for (int64_t id : G.ids) {
            Req &r = s->reqs[id];
            advance(s, r);
            if (r.state == Q_DONE) {
                if (r.x_out && r.n > 0) {
                    if (!hip_ok(hipMemcpyAsync(r.x_out, s->pool + r.off + r.L.x, sizeof(double) * 4 * (size_t)r.n,
                                               hipMemcpyDeviceToDevice, st),
                                "serve x copy"))
                        return ABILU_EDEVICE;
                    copied = true;
                }
                done.push_back(id);
            }
        }
    if (copied && !hip_ok(hipStreamSynchronize(st), "serve x copy sync")) return ABILU_EDEVICE;
    const double t = now_s() - s->t0;
    for (int64_t id : done) {
        Req &r = s->reqs[id];
        r.res.t_done = t;
        release(s, r);
        ++s->stat_retired;
    }
    return ABILU_OK;
}

abilu_status submit_impl(abilu_server *s, const abilu_request *q, double arrival, int64_t *id) {
    Req r;
    r.spec = q->gen;
    r.x_out = q->d_x_out;
    r.arrival = arrival;
    r.res.t_arrival = arrival;
    const int64_t my = (int64_t)s->reqs.size();
    if (id) *id = my;
    int32_t n = 0;
    int64_t Z = 0;
    if (abilu_gen_sizes(&r.spec, &n, &Z) != ABILU_OK) {
        r.state = Q_DONE;
        r.res.status = ABILU_EINVAL;
        r.res.t_done = arrival;
        s->reqs.push_back(r);
        return ABILU_OK;
    }
    r.n = n;
    r.Z = Z;
    r.L = req_layout(s->cfg, n, Z, abilu_gen_scratch_bytes(&r.spec));
    r.res.n = n;
    r.res.nnzb = Z;
    r.res.footprint_bytes = (int64_t)r.L.total;
    if (r.L.total > s->alloc.size) {
        r.state = Q_DONE;
        r.res.status = ABILU_ENOMEM;
        r.res.t_done = arrival;
        s->reqs.push_back(r);
        return ABILU_OK;
    }
    s->reqs.push_back(r);
    s->queue.push_back(my);
    return ABILU_OK;
}

int count_active(const abilu_server *s) {
    int a = 0;
    for (int q = 0; q < s->cfg.max_active; ++q) a += s->slot_req[q] >= 0;
    return a;
}

void free_server(abilu_server *s) {
    if (!s) return;
    if (s->setup) (void)hipStreamSynchronize(s->setup);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    if (s->setup) (void)hipStreamDestroy(s->setup);
    (void)hipFree(s->d_slots);
    (void)hipFree(s->d_tab);
    (void)hipFree(s->d_hdr);
    if (s->h_slots) (void)hipHostFree(s->h_slots);
    if (s->h_tab) (void)hipHostFree(s->h_tab);
    if (s->h_hdr) (void)hipHostFree(s->h_hdr);
    (void)hipFree(s->d_sdesc);
    (void)hipFree(s->d_sslot);
    (void)hipFree(s->d_stab);
    (void)hipFree(s->d_adm);
    if (s->h_sdesc) (void)hipHostFree(s->h_sdesc);
    if (s->h_stab) (void)hipHostFree(s->h_stab);
    if (s->h_adm) (void)hipHostFree(s->h_adm);
    delete s;
}

}  // namespace

extern "C" size_t abilu_serve_footprint(const abilu_serve_config *cfg, const abilu_gen_spec *spec) {
    if (!config_ok(cfg) || !spec) return 0;
    int32_t n = 0;
    int64_t Z = 0;
    if (abilu_gen_sizes(spec, &n, &Z) != ABILU_OK) return 0;
    return req_layout(*cfg, n, Z, abilu_gen_scratch_bytes(spec)).total;
}

extern "C" abilu_status abilu_serve_create(const abilu_serve_config *cfg, void *d_pool, size_t pool_bytes,
                                           abilu_server **out) {
    if (!out) return ABILU_EINVAL;
    *out = nullptr;
    if (!config_ok(cfg) || cfg->reserved != 0 || !d_pool || pool_bytes < 256 || ((uintptr_t)d_pool & 255))
        return ABILU_EINVAL;
    abilu_server *s = new abilu_server();
    s->cfg = *cfg;
    s->pool = (char *)d_pool;
    s->alloc.init(pool_bytes);
    const int S = cfg->max_active;
    s->tab_cap = 3 * SH_COUNT * S;
    s->slot_req.assign(S, -1);
    s->ev.assign(S, nullptr);
    s->t0 = now_s();
    bool ok = hip_ok(hipGetDevice(&s->device), "hipGetDevice") &&
              hip_ok(hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking), "serve setup stream") &&
              hip_ok(hipMalloc(&s->d_slots, sizeof(Slot) * S), "serve slots") &&
              hip_ok(hipMalloc(&s->d_tab, sizeof(Member) * s->tab_cap), "serve tables") &&
              hip_ok(hipMalloc(&s->d_hdr, (size_t)HDR * S), "serve headers") &&
              hip_ok(hipHostMalloc((void **)&s->h_slots, sizeof(Slot) * S, hipHostMallocDefault), "serve pinned") &&
              hip_ok(hipHostMalloc((void **)&s->h_tab, sizeof(Member) * s->tab_cap, hipHostMallocDefault),
                     "serve pinned") &&
              hip_ok(hipHostMalloc((void **)&s->h_hdr, (size_t)HDR * S, hipHostMallocDefault), "serve pinned") &&
              hip_ok(hipMalloc(&s->d_sdesc, sizeof(SetupDesc) * S), "serve setup descriptors") &&
              hip_ok(hipMalloc(&s->d_sslot, sizeof(Slot) * S), "serve staged slots") &&
              hip_ok(hipMalloc(&s->d_stab, sizeof(Member) * SS_COUNT * S), "serve setup tables") &&
              hip_ok(hipMalloc(&s->d_adm, sizeof(int64_t) * 4 * S), "serve admission words") &&
              hip_ok(hipHostMalloc((void **)&s->h_sdesc, sizeof(SetupDesc) * S, hipHostMallocDefault), "serve pinned") &&
              hip_ok(hipHostMalloc((void **)&s->h_stab, sizeof(Member) * SS_COUNT * S, hipHostMallocDefault),
                     "serve pinned") &&
              hip_ok(hipHostMalloc((void **)&s->h_adm, sizeof(int64_t) * 4 * S, hipHostMallocDefault), "serve pinned");
    for (int q = 0; ok && q < S; ++q)
        ok = hip_ok(hipEventCreateWithFlags(&s->ev[q], hipEventDisableTiming), "serve events");
    if (ok) ok = hip_ok(hipMemset(s->d_hdr, 0, (size_t)HDR * S), "serve header init");
    if (!ok) {
        free_server(s);
        return ABILU_EDEVICE;
    }
    *out = s;
    return ABILU_OK;
}

extern "C" abilu_status abilu_serve_destroy(abilu_server *srv) {
    if (!srv) return ABILU_EINVAL;
    free_server(srv);
    return ABILU_OK;
}

extern "C" abilu_status abilu_serve_submit(abilu_server *srv, const abilu_request *req, int64_t *id) {
    if (!srv || !req) return ABILU_EINVAL;
    return submit_impl(srv, req, now_s() - srv->t0, id);
}

extern "C" abilu_status abilu_serve_step(abilu_server *srv, void *stream, int32_t *active, int32_t *queued) {
    if (!srv) return ABILU_EINVAL;
    const abilu_status e = step_impl(srv, (hipStream_t)stream);
    if (active) *active = count_active(srv);
    if (queued) *queued = (int32_t)srv->queue.size();
    return e;
}

extern "C" abilu_status abilu_serve_poll(abilu_server *srv, int64_t id, int32_t *done, abilu_request_result *out) {
    if (!srv || !done || id < 0 || id >= (int64_t)srv->reqs.size()) return ABILU_EINVAL;
    const Req &r = srv->reqs[id];
    *done = r.state == Q_DONE ? 1 : 0;
    if (*done && out) *out = r.res;
    return ABILU_OK;
}

extern "C" abilu_status abilu_serve_run(abilu_server *srv, const abilu_request *reqs, int32_t count,
                                        abilu_request_result *results, double *elapsed_s, void *stream) {
    if (!srv || count < 0 || (count > 0 && (!reqs || !results))) return ABILU_EINVAL;
    for (int32_t q = 0; q < count; ++q)
        if (!(reqs[q].arrival_s >= 0.0)) return ABILU_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    // release order: by arrival time, ties by index
    std::vector<int32_t> order(count);
    for (int32_t q = 0; q < count; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
    const double start = now_s() - srv->t0;
    std::vector<int64_t> ids(count, -1);
    size_t next = 0;
    abilu_status e = ABILU_OK;
    int32_t remaining = count;
    std::vector<char> seen(count, 0);
    while (remaining > 0) {
        const double t = now_s() - srv->t0;
        while (next < order.size() && start + reqs[order[next]].arrival_s <= t) {
            const int32_t q = order[next++];
            if ((e = submit_impl(srv, &reqs[q], start + reqs[q].arrival_s, &ids[q])) != ABILU_OK) return e;
        }
        const bool idle = count_active(srv) == 0 && srv->queue.empty();
        if (idle && next < order.size()) {
            const double wait = start + reqs[order[next]].arrival_s - (now_s() - srv->t0);
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.01)));
            continue;
        }
        if ((e = step_impl(srv, st)) != ABILU_OK) return e;
        for (int32_t q = 0; q < count; ++q) {
            if (seen[q] || ids[q] < 0) continue;
            const Req &r = srv->reqs[ids[q]];
            if (r.state == Q_DONE) {
                results[q] = r.res;
                results[q].t_arrival -= start;
                results[q].t_admit = r.res.t_admit > 0 ? r.res.t_admit - start : 0.0;
                results[q].t_done -= start;
                seen[q] = 1;
                --remaining;
            }
        }
    }
    if (elapsed_s) *elapsed_s = now_s() - srv->t0 - start;
    return ABILU_OK;
}

extern "C" abilu_status abilu_serve_stats(const abilu_server *srv, abilu_serve_stats_t *out) {
    if (!srv || !out) return ABILU_EINVAL;
    out->ticks = srv->stat_ticks;
    out->launches = srv->stat_launches;
    out->admitted = srv->stat_admitted;
    out->retired = srv->stat_retired;
    out->bytes = srv->stat_bytes;
    return ABILU_OK;
}
