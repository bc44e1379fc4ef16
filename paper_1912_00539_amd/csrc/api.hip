// Library runtime: workspace layout, status strings, flag word, STREAM copy reference and
// per-launch event profiling.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "abilu_internal.h"

namespace abilu {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Workspace layout(const abilu_pattern *p, abilu_prec prec, int restart) {
    Workspace W{};
    const size_t sf = (prec == ABILU_F32) ? 4 : 8;
    const size_t n = (size_t)p->n, Z = (size_t)p->nnzb, nv = 4 * n;
    const int m = restart > 0 ? restart : 0;
    W.restart = m;
    W.nb_vec = div_up((int64_t)(nv > 0 ? nv : 1), VEC_TILE);
    size_t o = 0;
    W.flags = 0;
    W.status = 64;                      // 8 doubles at byte 64..127
    o = 256;
    W.x2 = o; o = align256(o + Z * 16 * sf);
    W.d2 = o; o = align256(o + n * 16 * sf);
    W.ya = o; o = align256(o + nv * sf);
    W.yb = o; o = align256(o + nv * sf);
    W.za = o; o = align256(o + nv * sf);
    W.zb = o; o = align256(o + nv * sf);
    W.partials = o; o = align256(o + sizeof(double) * (size_t)(m + 2) * W.nb_vec);
    W.hess = o; o = align256(o + sizeof(double) * (size_t)(m + 1) * (m > 0 ? m : 1));
    W.cs = o; o = align256(o + sizeof(double) * (m + 2));
    W.sn = o; o = align256(o + sizeof(double) * (m + 2));
    W.g = o; o = align256(o + sizeof(double) * (m + 2));
    W.coef = o; o = align256(o + sizeof(double) * (m + 2));
    W.misc = o; o = align256(o + sizeof(double) * 16);
    W.red = o; o = align256(o + sizeof(double) * (m + 4));
    if (m > 0) {
        W.V = o; o = align256(o + sizeof(double) * (size_t)(m + 1) * nv);
        W.Z = o; o = align256(o + sizeof(double) * (size_t)m * nv);
    } else {
        W.V = W.Z = o;
    }
    W.total = o;
    return W;
}

namespace {
thread_local char g_last_error[512] = "";
}

bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    snprintf(g_last_error, sizeof g_last_error, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return false;
}

void note_error(const char *what) { snprintf(g_last_error, sizeof g_last_error, "%s", what); }

abilu_status launch_status() { return hip_ok(hipGetLastError(), "kernel launch") ? ABILU_OK : ABILU_EDEVICE; }

// ------------------------------------------------------------------ profiling
namespace {
struct Prof {
    bool on = false;
    int cap = 0, used = 0, dropped = 0;
    std::vector<hipEvent_t> ev;      // 2 per slot
    std::vector<int> name_of_slot;
    std::vector<double> bytes_of_slot;
    std::vector<std::string> names;
};
Prof g_prof;

int name_id(const char *name) {
    for (size_t q = 0; q < g_prof.names.size(); ++q)
        if (g_prof.names[q] == name) return (int)q;
    g_prof.names.emplace_back(name);
    return (int)g_prof.names.size() - 1;
}
}  // namespace

ProfScope::ProfScope(const char *name, hipStream_t s, double bytes) : slot(-1), stream(s) {
    if (!g_prof.on) return;
    if (g_prof.used >= g_prof.cap) { ++g_prof.dropped; return; }
    slot = g_prof.used++;
    g_prof.name_of_slot[slot] = name_id(name);
    g_prof.bytes_of_slot[slot] = bytes;
    (void)hipEventRecord(g_prof.ev[2 * slot], s);
}

int prof_mark() { return g_prof.on ? g_prof.used : 0; }

void prof_add_bytes(int slot, double delta) {
    if (g_prof.on && slot >= 0 && slot < g_prof.used) g_prof.bytes_of_slot[slot] += delta;
}

void prof_cancel_bytes(int from, int to) {
    if (!g_prof.on) return;
    for (int q = from; q < to && q < g_prof.used; ++q) g_prof.bytes_of_slot[q] = 0.0;
}

ProfScope::~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], stream);
}

}  // namespace abilu

using namespace abilu;

extern "C" abilu_status abilu_profile_enable(int32_t enable, int32_t max_launches) {
    if (!enable) { g_prof.on = false; return ABILU_OK; }
    if (max_launches < 1) return ABILU_EINVAL;
    if ((int)g_prof.ev.size() < 2 * max_launches) {
        size_t old = g_prof.ev.size();
        g_prof.ev.resize(2 * (size_t)max_launches);
        for (size_t q = old; q < g_prof.ev.size(); ++q)
            if (!hip_ok(hipEventCreate(&g_prof.ev[q]), "hipEventCreate")) return ABILU_EDEVICE;
    }
    g_prof.name_of_slot.assign(max_launches, -1);
    g_prof.bytes_of_slot.assign(max_launches, 0.0);
    g_prof.cap = max_launches;
    g_prof.used = 0;
    g_prof.dropped = 0;
    g_prof.on = true;
    return ABILU_OK;
}

extern "C" abilu_status abilu_profile_report(char *buf, size_t len) {
    if (!buf || len == 0) return ABILU_EINVAL;
    std::vector<double> ms(g_prof.names.size(), 0.0), by(g_prof.names.size(), 0.0);
    std::vector<int> cnt(g_prof.names.size(), 0);
    for (int q = 0; q < g_prof.used; ++q) {
        if (!hip_ok(hipEventSynchronize(g_prof.ev[2 * q + 1]), "profile event sync")) return ABILU_EDEVICE;
        float t = 0.f;
        if (!hip_ok(hipEventElapsedTime(&t, g_prof.ev[2 * q], g_prof.ev[2 * q + 1]), "profile elapsed")) return ABILU_EDEVICE;
        ms[g_prof.name_of_slot[q]] += t;
        by[g_prof.name_of_slot[q]] += g_prof.bytes_of_slot[q];
        cnt[g_prof.name_of_slot[q]] += 1;
    }
    std::string s = "{";
    char tmp[256];
    bool first = true;
    for (size_t q = 0; q < g_prof.names.size(); ++q) {
        if (!cnt[q]) continue;
        snprintf(tmp, sizeof tmp, "%s\"%s\": [%d, %.6f, %.0f]", first ? "" : ", ", g_prof.names[q].c_str(), cnt[q],
                 ms[q], by[q]);
        s += tmp;
        first = false;
    }
    snprintf(tmp, sizeof tmp, "%s\"_dropped\": [%d, 0.0, 0]}", first ? "" : ", ", g_prof.dropped);
    s += tmp;
    strncpy(buf, s.c_str(), len - 1);
    buf[len - 1] = 0;
    return ABILU_OK;
}

// ------------------------------------------------------------------ status, workspace, flags
extern "C" abilu_status abilu_last_error(char *buf, size_t len) {
    if (!buf || len == 0) return ABILU_EINVAL;
    strncpy(buf, g_last_error, len - 1);
    buf[len - 1] = 0;
    return ABILU_OK;
}

extern "C" const char *abilu_status_string(abilu_status s) {
    switch (s) {
        case ABILU_OK: return "ok";
        case ABILU_WARN_MODIFIED: return "warning: singular diagonal block replaced by identity";
        case ABILU_WARN_NOCONV: return "warning: FGMRES did not converge within maxit";
        case ABILU_EINVAL: return "error: invalid argument";
        case ABILU_EPATTERN: return "error: invalid block pattern";
        case ABILU_ENOMEM: return "error: allocation failed";
        case ABILU_EDEVICE: return "error: HIP runtime or kernel launch failure";
        case ABILU_ENONFINITE: return "error: non-finite value";
    }
    return "unknown status";
}

extern "C" size_t abilu_workspace_bytes(const abilu_pattern *p, abilu_prec prec, int32_t fgmres_restart) {
    if (!p || (prec != ABILU_F32 && prec != ABILU_F64) || fgmres_restart < 0) return 0;
    return layout(p, prec, fgmres_restart).total;
}

namespace {
__global__ void k_fill_u32(unsigned *p, unsigned v) { *p = v; }
}  // namespace

extern "C" abilu_status abilu_clear_flags(void *d_work, void *stream) {
    if (!d_work) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    ProfScope ps("clear_flags", s);
    k_fill_u32<<<1, 1, 0, s>>>((unsigned *)d_work, 0u);
    return launch_status();
}

extern "C" abilu_status abilu_read_flags(void *d_work, int32_t clear, uint32_t *h_flags, void *stream) {
    if (!d_work || !h_flags) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    uint32_t v = 0;
    if (!hip_ok(hipMemcpyAsync(&v, d_work, sizeof v, hipMemcpyDeviceToHost, s), "read flags copy")) return ABILU_EDEVICE;
    if (!hip_ok(hipStreamSynchronize(s), "read flags sync")) return ABILU_EDEVICE;
    *h_flags = v;
    if (clear) return abilu_clear_flags(d_work, stream);
    return ABILU_OK;
}

// ------------------------------------------------------------------ STREAM copy
namespace {
constexpr int COPY_E = 4;   // float4 per thread
__global__ __launch_bounds__(WG) void k_stream_copy(int64_t n16, const float4 *__restrict__ src,
                                                    float4 *__restrict__ dst) {
    int64_t base = (int64_t)blockIdx.x * WG * COPY_E + threadIdx.x;
    float4 v[COPY_E];
#pragma unroll
    for (int q = 0; q < COPY_E; ++q) {
        int64_t t = base + (int64_t)q * WG;
        if (t < n16) v[q] = src[t];
    }
#pragma unroll
    for (int q = 0; q < COPY_E; ++q) {
        int64_t t = base + (int64_t)q * WG;
        if (t < n16) dst[t] = v[q];
    }
}
}  // namespace

extern "C" abilu_status abilu_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *stream) {
    if ((bytes % 16) || ((uintptr_t)d_dst % 16) || ((uintptr_t)d_src % 16)) return ABILU_EINVAL;
    if (bytes == 0) return ABILU_OK;
    if (!d_dst || !d_src) return ABILU_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t n16 = (int64_t)(bytes / 16);
    ProfScope ps("stream_copy", s, 2.0 * (double)bytes);
    k_stream_copy<<<div_up(n16, (int64_t)WG * COPY_E), WG, 0, s>>>(n16, (const float4 *)d_src, (float4 *)d_dst);
    return launch_status();
}
