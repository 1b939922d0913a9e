// Host side of the C ABI declared in include/ptp.h: plans, workspace carve,
// launches and status reporting.  No allocation happens here: every device
// buffer comes from the caller.
#include <stdio.h>
#include <string.h>

#include <string>

#include "ptp.h"
#include "ptp_device.h"
#include "ptp_kernels.h"

using namespace ptp;

struct ptp_plan {
    int n = 0, f = 0, m = 0;
    ptp_options opt{};
    int device = 0, cus = 0;
    int g_bfs = 0, g_run = 0, gmax = 0, max_run = 0;
    int g_used = 0;
    Layout layout{};
    Work work{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    const int32_t* S = nullptr;
    int rho = 0, reach = 0;
    bool prepared = false;
    bool ran = false;
    int h_ctrl[C_WORDS];
    std::string err;
};

namespace {

ptp_status fail(ptp_plan* p, ptp_status s, const std::string& msg) {
    if (p) p->err = msg;
    return s;
}

ptp_status hip_fail(ptp_plan* p, hipError_t e, const char* what) {
    return fail(p, PTP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace ptp {

size_t work_layout(int n, int f, int gmax, Layout* L) {
    const size_t N = (size_t)n, Fc = 3 * (size_t)f;
    const size_t nwords = (N + 31) / 32;
    const size_t scan_blocks = (N + 1 + 4095) / 4096 + 1;
    const size_t sizes[kLayoutParts] = {
        sizeof(int) * C_WORDS,      // ctrl
        sizeof(int) * N,            // level
        sizeof(int) * N,            // perm
        sizeof(int) * N,            // iperm
        sizeof(int) * (N + 2),      // offsets
        sizeof(int) * (N + 1),      // rowO
        sizeof(int) * (Fc + 1),     // faceO
        sizeof(int) * N,            // cursor
        sizeof(int) * (N + 1),      // rowN
        sizeof(int2) * (Fc + 1),    // wedge
        sizeof(float4) * N,         // xyz
        sizeof(float) * 2 * N,      // dist
        sizeof(int) * 2 * N,        // lab
        sizeof(unsigned) * 2 * nwords,
        sizeof(int) * 4 * (size_t)gmax,
        sizeof(int) * N,            // retire
        sizeof(int) * scan_blocks,  // scan_tmp
        sizeof(unsigned) * kLine * ((size_t)gmax + 1),   // barrier lines
    };
    size_t off = 0;
    for (int i = 0; i < kLayoutParts; ++i) {
        L->off[i] = off;
        off += align_up(sizes[i]);
    }
    L->total = off;
    return off;
}

Work carve(void* base, int, int, int, const Layout& L) {
    char* b = static_cast<char*>(base);
    Work w;
    w.ctrl = reinterpret_cast<int*>(b + L.off[0]);
    w.level = reinterpret_cast<int*>(b + L.off[1]);
    w.perm = reinterpret_cast<int*>(b + L.off[2]);
    w.iperm = reinterpret_cast<int*>(b + L.off[3]);
    w.offsets = reinterpret_cast<int*>(b + L.off[4]);
    w.rowO = reinterpret_cast<int*>(b + L.off[5]);
    w.faceO = reinterpret_cast<int*>(b + L.off[6]);
    w.cursor = reinterpret_cast<int*>(b + L.off[7]);
    w.rowN = reinterpret_cast<int*>(b + L.off[8]);
    w.wedge = reinterpret_cast<int2*>(b + L.off[9]);
    w.xyz = reinterpret_cast<float4*>(b + L.off[10]);
    w.dist = reinterpret_cast<float*>(b + L.off[11]);
    w.lab = reinterpret_cast<int*>(b + L.off[12]);
    w.bits = reinterpret_cast<unsigned*>(b + L.off[13]);
    w.cnt = reinterpret_cast<int*>(b + L.off[14]);
    w.retire = reinterpret_cast<int*>(b + L.off[15]);
    w.scan_tmp = reinterpret_cast<int*>(b + L.off[16]);
    w.bar = reinterpret_cast<unsigned*>(b + L.off[17]);
    return w;
}

}  // namespace ptp

extern "C" {

const char* ptp_version(void) { return "ptp-mi355x 0.1 (gfx950)"; }

ptp_status ptp_plan_create(ptp_plan** out, int32_t n, int32_t f, int32_t m, const ptp_options* opt) {
    if (!out) return PTP_EINVAL;
    *out = nullptr;
    if (n < 1 || f < 0 || m < 1 || m > n) return PTP_EINVAL;
    if (n > (1 << 29) || (long long)f * 3 >= (1ll << 31)) return PTP_EUNSUPPORTED;
    ptp_options o;
    if (opt) {
        o = *opt;
    } else {
        o.tol = 1e-3f;
        o.max_iters = 0;
        o.window = 0;
        o.want_labels = 0;
        o.workgroups = 0;
    }
    if (!(o.tol > 0.f) || o.max_iters < 0 || o.window < 0 || o.workgroups < 0) return PTP_EINVAL;
    ptp_plan* p = new (std::nothrow) ptp_plan();
    if (!p) return PTP_ENOMEM;
    p->n = n;
    p->f = f;
    p->m = m;
    p->opt = o;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
    int coop = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, p->device);
    if (e != hipSuccess || !coop || p->cus < 1) {
        delete p;
        return PTP_EDEVICE;
    }
    const bool labels = o.want_labels != 0;
    const int max_bfs = max_coop_blocks_bfs(p->cus);
    const int max_run = max_coop_blocks_run(p->cus, labels);
    p->g_bfs = p->cus < max_bfs ? p->cus : max_bfs;
    p->max_run = max_run;
    // an explicit grid is fixed here; the automatic one is chosen per prepared
    // mesh in ptp_run, so the barrier lines cover the largest possible grid
    p->g_run = o.workgroups > 0 ? (o.workgroups < max_run ? o.workgroups : max_run) : 0;
    p->gmax = p->g_bfs > max_run ? p->g_bfs : max_run;
    work_layout(n, f, p->gmax, &p->layout);
    *out = p;
    return PTP_OK;
}

ptp_status ptp_workspace_bytes(const ptp_plan* p, size_t* bytes) {
    if (!p || !bytes) return PTP_EINVAL;
    *bytes = p->layout.total;
    return PTP_OK;
}

ptp_status ptp_prepare(ptp_plan* p, const float* dV, const int32_t* dF, const int32_t* dS,
                       void* dWork, size_t work_bytes, void* stream) {
    if (!p) return PTP_EINVAL;
    p->prepared = false;
    p->ran = false;
    if (!dV || !dS || (!dF && p->f > 0) || !dWork)
        return fail(p, PTP_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(dWork) & 255)
        return fail(p, PTP_EINVAL, "workspace must be 256-byte aligned");
    if (work_bytes < p->layout.total)
        return fail(p, PTP_ENOMEM, "workspace smaller than ptp_workspace_bytes()");
    p->ws = dWork;
    p->ws_bytes = work_bytes;
    p->stream = static_cast<hipStream_t>(stream);
    p->work = carve(dWork, p->n, p->f, p->gmax, p->layout);
    p->S = dS;
    hipError_t e = launch_prepare(p->work, p->n, p->f, p->m, dV, dF, dS, p->g_bfs, p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "prepare launch");
    e = hipMemcpyAsync(p->h_ctrl, p->work.ctrl, sizeof(int) * 8, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "prepare");
    const int st = p->h_ctrl[C_STATUS];
    if (p->h_ctrl[C_ABORT]) return fail(p, PTP_EDEVICE, "BFS barrier timed out");
    if (st) {
        std::string msg = "invalid input:";
        if (st & ST_BAD_FACE) msg += " face index out of range;";
        if (st & ST_BAD_COORD) msg += " non-finite coordinate;";
        if (st & ST_BAD_SOURCE) msg += " source index out of range;";
        if (st & ST_DUP_SOURCE) msg += " duplicate source;";
        return fail(p, PTP_EINVAL, msg);
    }
    p->rho = p->h_ctrl[C_RHO];
    p->reach = p->h_ctrl[C_REACH];
    if (p->rho < 1 || p->reach < p->m || p->reach > p->n)
        return fail(p, PTP_EDEVICE, "BFS produced an inconsistent result");
    p->prepared = true;
    return PTP_OK;
}

ptp_status ptp_run(ptp_plan* p, float* dDist, int32_t* dLabel, void* stream) {
    if (!p) return PTP_EINVAL;
    if (!p->prepared) return fail(p, PTP_EINVAL, "ptp_run before a successful ptp_prepare");
    if (!dDist) return fail(p, PTP_EINVAL, "null distance output");
    const bool labels = p->opt.want_labels != 0;
    if (labels && !dLabel) return fail(p, PTP_EINVAL, "plan wants labels: null label output");
    p->stream = static_cast<hipStream_t>(stream);
    RunParams rp;
    rp.n = p->n;
    rp.m = p->m;
    rp.rho = p->rho;
    rp.kmax = p->opt.max_iters > 0 ? p->opt.max_iters : 4 * p->rho + 16;
    rp.window = p->opt.window;
    rp.tol = p->opt.tol;
    rp.S = p->S;
    rp.out_d = dDist;
    rp.out_l = labels ? dLabel : nullptr;
    // Automatic grid: about one workgroup (256 threads) per 1024 reachable
    // vertices, within [16, 512] and the co-residency limit.  Measured on the
    // icosphere workloads: the per-iteration cost is flat from ~n/2048 to
    // ~n/512 workgroups and rises outside.
    int g = p->g_run;
    if (g <= 0) {
        g = p->reach / 1024;
        if (g < 16) g = 16;
        if (g > 512) g = 512;
        if (g > p->max_run) g = p->max_run;
    }
    p->g_used = g;
    hipError_t e = launch_run(p->work, rp, labels, g, p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "run launch");
    p->ran = true;
    return PTP_OK;
}

ptp_status ptp_get_stats(ptp_plan* p, ptp_stats* st) {
    if (!p) return PTP_EINVAL;
    if (!p->ran) return fail(p, PTP_EINVAL, "no run to report");
    hipError_t e = hipMemcpyAsync(p->h_ctrl, p->work.ctrl, sizeof(int) * 8, hipMemcpyDeviceToHost,
                                  p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "stats");
    if (st) {
        st->iterations = p->h_ctrl[C_ITERS];
        st->n_toplesets = p->rho;
        st->reachable = p->reach;
        st->workgroups = p->g_used;
        st->vertex_updates = ((int64_t)(uint32_t)p->h_ctrl[C_UPD_HI] << 32) |
                             (int64_t)(uint32_t)p->h_ctrl[C_UPD_LO];
    }
    if (p->h_ctrl[C_ABORT]) return fail(p, PTP_EDEVICE, "relaxation barrier timed out");
    if (p->h_ctrl[C_RUNSTAT]) return fail(p, PTP_ENOCONV, "iteration cap reached");
    return PTP_OK;
}

ptp_status ptp_solve(ptp_plan* p, const float* dV, const int32_t* dF, const int32_t* dS,
                     void* dWork, size_t work_bytes, float* dDist, int32_t* dLabel,
                     ptp_stats* stats, void* stream) {
    ptp_status s = ptp_prepare(p, dV, dF, dS, dWork, work_bytes, stream);
    if (s != PTP_OK) return s;
    s = ptp_run(p, dDist, dLabel, stream);
    if (s != PTP_OK) return s;
    return ptp_get_stats(p, stats);
}

ptp_status ptp_get_order(ptp_plan* p, int32_t* dPerm, int32_t* dOffsets, void* stream) {
    if (!p) return PTP_EINVAL;
    if (!p->prepared) return fail(p, PTP_EINVAL, "no prepared mesh");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (dPerm)
        e = hipMemcpyAsync(dPerm, p->work.perm, sizeof(int) * (size_t)p->n,
                           hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && dOffsets)
        e = hipMemcpyAsync(dOffsets, p->work.offsets, sizeof(int) * ((size_t)p->rho + 1),
                           hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(p, e, "get_order");
    return PTP_OK;
}

ptp_status ptp_get_schedule(ptp_plan* p, int32_t* hRetire) {
    if (!p || !hRetire) return PTP_EINVAL;
    if (!p->ran) return fail(p, PTP_EINVAL, "no run to report");
    hipError_t e = hipMemcpyAsync(hRetire, p->work.retire, sizeof(int) * (size_t)p->rho,
                                  hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "get_schedule");
    return PTP_OK;
}

int32_t ptp_n_toplesets(const ptp_plan* p) { return p && p->prepared ? p->rho : -1; }

const char* ptp_last_error(const ptp_plan* p) { return p ? p->err.c_str() : "null plan"; }

void ptp_plan_destroy(ptp_plan* p) { delete p; }

}  // extern "C"
