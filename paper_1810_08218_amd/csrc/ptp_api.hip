// Host side of the C ABI declared in include/ptp.h: plans (one mesh) and
// batches (many meshes) share one implementation, the batch; a plan is a
// batch of one.  The host validates sizes, carves the caller's workspace,
// builds the work distribution of the persistent launches (groups of
// workgroups, longest-processing-time assignment of meshes to groups),
// launches, and reports per-mesh status.  No device allocation happens here.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "ptp.h"
#include "ptp_device.h"
#include "ptp_kernels.h"
#include "ptp_mlp.h"

using namespace ptp;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Work distribution of one persistent launch.
struct Sched {
    int G = 0;
    int ngroups = 0;
    std::vector<WgInfo> wg;      // [G]
    std::vector<int> glist;      // starts [ngroups + 1] (absolute), then mesh ids
    std::vector<int> gsize_of;   // [B] group size of each mesh's class
    // the same assignment as queues the groups take meshes from at run time:
    // [4] starts of the class lists (small, medium, large) and their end,
    // [ngroups] class of each group, then the class lists, each ordered by
    // decreasing estimated time
    std::vector<int> queue;
};

// Seconds of the BFS of a mesh of n vertices and rho toplesets on a group of
// s workgroups: a level costs a group barrier and a few round trips.  Only
// the relative size matters: it drives the assignment, the results never
// depend on it.
double est_time(long long n, long long rho, int s) {
    return (double)rho * 5e-6 + 4.0 * (double)n * 8e-9 / (double)s;
}

// Relaxation time of a mesh with K iterations and U vertex updates on a
// group of s workgroups, from measured runs on the 512-mesh batch: a group
// iteration costs ~1.6 us on one workgroup and ~6.5 us on several (barrier,
// controller), and a thread takes ~3 us per band vertex it owns.  Without a
// measured run, K ~ 1.2 rho and U ~ 0.2 n rho stand in.
double est_run(double K, double U, int s) {
    return K * (s == 1 ? 1.6e-6 : 6.5e-6) + 3e-6 * U / (256.0 * s);
}

using CostFn = std::function<double(int, int)>;   // (mesh, group size) -> seconds

Sched make_schedule(const std::vector<MeshDesc>& mesh, const CostFn& est, const ptp_schedule& p, int gmax,
                    bool single, int single_g) {
    Sched s;
    const int B = (int)mesh.size();
    s.gsize_of.assign(B, 1);
    std::vector<std::vector<int>> groups;
    std::vector<int> gsz, gclass;
    std::vector<int> qlists[3];
    if (single) {
        groups.push_back({0});
        gsz.push_back(std::max(1, std::min(single_g, gmax)));
        gclass.push_back(0);
        qlists[0] = {0};
        s.gsize_of[0] = gsz[0];
    } else {
        const int G = std::max(1, std::min(p.workgroups, gmax));
        int size_c[3] = {1, std::max(1, p.medium_group), std::max(1, p.large_group)};
        std::vector<int> members[3];
        for (int b = 0; b < B; ++b) {
            const int n = mesh[b].n;
            members[n < p.small_limit ? 0 : (n < p.large_limit ? 1 : 2)].push_back(b);
        }
        for (int c = 0; c < 3; ++c) size_c[c] = std::min(size_c[c], G);
        // every non-empty class gets one group, largest meshes first; a class
        // that no longer fits joins the single-workgroup class
        int ng[3] = {0, 0, 0};
        int used = 0;
        for (int c = 2; c >= 1; --c) {
            if (members[c].empty()) continue;
            if (used + size_c[c] + (members[0].empty() ? 0 : 1) > G) {
                members[0].insert(members[0].end(), members[c].begin(), members[c].end());
                members[c].clear();
                continue;
            }
            ng[c] = 1;
            used += size_c[c];
        }
        if (!members[0].empty()) {
            ng[0] = 1;
            used += 1;
        }
        // each mesh's estimate at its class's group size, computed once
        std::vector<double> cost(B, 0.0);
        double C[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c)
            for (int b : members[c]) {
                cost[b] = est(b, size_c[c]);
                C[c] += cost[b];
            }
        // hand out the remaining workgroups to the class with the largest load per group
        for (;;) {
            int best = -1;
            double bl = 0;
            for (int c = 0; c < 3; ++c) {
                if (members[c].empty() || ng[c] >= (int)members[c].size()) continue;
                if (used + size_c[c] > G) continue;
                const double load = C[c] / ng[c];
                if (load > bl) {
                    bl = load;
                    best = c;
                }
            }
            if (best < 0) break;
            ng[best] += 1;
            used += size_c[best];
        }
        // longest processing time first inside each class
        for (int c = 2; c >= 0; --c) {
            if (members[c].empty()) continue;
            std::vector<int> ord = members[c];
            const int sc = size_c[c];
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
            qlists[c] = ord;
            const int first = (int)groups.size();
            for (int g = 0; g < ng[c]; ++g) {
                groups.emplace_back();
                gsz.push_back(sc);
                gclass.push_back(c);
            }
            using Item = std::pair<double, int>;
            std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
            for (int g = 0; g < ng[c]; ++g) heap.push({0.0, first + g});
            for (int b : ord) {
                Item it = heap.top();
                heap.pop();
                groups[it.second].push_back(b);
                it.first += cost[b];
                heap.push(it);
                s.gsize_of[b] = sc;
            }
        }
    }
    s.ngroups = (int)groups.size();
    s.glist.assign(s.ngroups + 1, 0);
    int pos = s.ngroups + 1;
    for (int g = 0; g < s.ngroups; ++g) {
        s.glist[g] = pos;
        pos += (int)groups[g].size();
    }
    s.glist[s.ngroups] = pos;
    for (int g = 0; g < s.ngroups; ++g)
        for (int b : groups[g]) s.glist.push_back(b);
    s.queue.assign(4, 0);
    for (int c = 0; c < 3; ++c) s.queue[c + 1] = s.queue[c] + (int)qlists[c].size();
    for (int g = 0; g < s.ngroups; ++g) s.queue.push_back(gclass[g]);
    for (int c = 0; c < 3; ++c) s.queue.insert(s.queue.end(), qlists[c].begin(), qlists[c].end());
    // Workgroup slots.  Consecutive launch indices go to the 8 XCDs in turn
    // (index i runs on XCD i mod 8), and each XCD has its own L2, so a group
    // placed on one XCD exchanges its data and barrier lines through one L2.
    // That pays for groups of up to kXcdGroup workgroups (one per CU of the
    // XCD; measured ~7% per iteration at 16-32); larger groups need the CUs
    // of every XCD and are spread evenly, in blocks of consecutive ranks per
    // XCD: consecutive ranks own consecutive positions, and a vertex's
    // neighbours sit in the same or adjacent toplesets, so most of the
    // distances a workgroup reads were written on its own XCD (measured
    // 8% less time per iteration on the level-7 icosphere than ranks dealt
    // round-robin).  Groups are placed largest first onto the XCD with the
    // most free slots.  Unused indices idle.
    std::vector<int> firsts(s.ngroups);
    int first = 0;
    for (int g = 0; g < s.ngroups; ++g) {
        firsts[g] = first;
        first += gsz[g];
    }
    if (!p.xcd_pack || s.ngroups == 0) {
        for (int g = 0; g < s.ngroups; ++g)
            for (int r = 0; r < gsz[g]; ++r) s.wg.push_back(WgInfo{g, r, gsz[g], firsts[g]});
        s.G = first;
        return s;
    }
    constexpr int kXcd = 8;
    const int cap = std::max(1, gmax / kXcd);
    const int xcd_group = p.xcd_pack > 1 ? p.xcd_pack : 32;
    int used[kXcd] = {0, 0, 0, 0, 0, 0, 0, 0};
    std::vector<int> ord(s.ngroups);
    for (int g = 0; g < s.ngroups; ++g) ord[g] = g;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return gsz[x] > gsz[y]; });
    std::vector<WgInfo> slot;      // by launch index
    // Every XCD holds at most `cap` workgroups, so launch indices stay below
    // 8 cap <= gmax.  A rank whose preferred XCD is full goes to the least
    // used one with room; if none has room, the placement falls back to
    // consecutive indices.
    bool full = false;
    auto put = [&](int x, const WgInfo& info) {
        if (used[x] >= cap) {
            int alt = -1;
            for (int y = 0; y < kXcd; ++y)
                if (used[y] < cap && (alt < 0 || used[y] < used[alt])) alt = y;
            if (alt < 0) {
                full = true;
                return;
            }
            x = alt;
        }
        const int idx = kXcd * used[x] + x;
        used[x] += 1;
        if ((int)slot.size() <= idx) slot.resize(idx + 1, WgInfo{-1, 0, 0, 0});
        slot[idx] = info;
    };
    for (int g : ord) {
        int best = 0;
        for (int x = 1; x < kXcd; ++x)
            if (used[x] < used[best]) best = x;
        if (gsz[g] <= xcd_group && used[best] + gsz[g] <= cap) {
            for (int r = 0; r < gsz[g]; ++r) put(best, WgInfo{g, r, gsz[g], firsts[g]});
        } else {
            // consecutive ranks (consecutive positions) on one XCD, in blocks
            for (int r = 0; r < gsz[g]; ++r) {
                const int x = (int)((long long)r * kXcd / gsz[g]);
                put(x, WgInfo{g, r, gsz[g], firsts[g]});
            }
        }
    }
    if (full || (int)slot.size() > gmax) {
        for (int g = 0; g < s.ngroups; ++g)
            for (int r = 0; r < gsz[g]; ++r) s.wg.push_back(WgInfo{g, r, gsz[g], firsts[g]});
        s.G = first;
        return s;
    }
    s.wg = slot;
    s.G = (int)slot.size();
    return s;
}

}  // namespace

namespace ptp {

size_t work_layout(const Sizes& z, Layout* L) {
    const size_t N = (size_t)z.N, F3 = 3 * (size_t)z.F, B = (size_t)z.B, G = (size_t)z.gmax;
    const size_t scan_blocks = (N + 1 + 4095) / 4096 + 1;
    const size_t sizes[kLayoutParts] = {
        sizeof(int) * C_WORDS,                 // ctrl
        sizeof(MeshDesc) * B,                  // mesh
        sizeof(MeshState) * B,                 // state
        sizeof(WgInfo) * G,                    // wg_prep
        sizeof(int) * (G + 8 + B),             // glist_prep
        sizeof(WgInfo) * G,                    // wg_run
        sizeof(int) * (G + 8 + B),             // glist_run
        sizeof(int) * (B + 1),                 // vo
        sizeof(int) * (B + 1),                 // fo3
        sizeof(int) * (B + 1),                 // so
        sizeof(int) * N,                       // level
        sizeof(int) * N,                       // perm
        sizeof(int) * N,                       // iperm
        sizeof(int) * (N + B + 1),             // offsets
        sizeof(int) * (N + 1),                 // rowO
        sizeof(int2) * (F3 + 1),               // wedgeO
        sizeof(int) * N,                       // cursor
        sizeof(int) * (N + 1),                 // fanlen
        sizeof(int) * (2 * F3 + 2),            // fanO
        sizeof(float4) * N,                    // xyz
        // dist / dl: one region, 8 bytes per entry.  A run uses either the
        // float double buffer (plain and warm runs) or the 8-byte one
        // (labelled runs: (distance, label) pairs; the float64 run: doubles)
        sizeof(unsigned long long) * 2 * N,    // dist and dl
        0,                                     // (dl aliases dist)
        sizeof(unsigned) * 2 * (size_t)z.W,    // bits
        sizeof(int) * 4 * G,                   // cnt
        sizeof(int) * N,                       // retire
        sizeof(int) * scan_blocks,             // scan_tmp
        sizeof(unsigned) * kLine * 2 * G,      // barrier lines
        sizeof(float4) * N,                    // feat
        sizeof(unsigned long long) * 2 * B,    // edge_acc (sums, maxima)
        sizeof(int) * B,                       // lds_mesh
        sizeof(int2) * N,                      // fanrow
        sizeof(int) * (2 * F3 + 1),            // fan
        sizeof(int) * kEll * N,                // ellO
        sizeof(WgInfo) * G,                    // wg_run64
        sizeof(int) * (G + 8 + B),             // glist_run64
        sizeof(double) * (size_t)z.S * (kCvtChunks * 6 + 4),   // cvt partial sums, centroids
        sizeof(int) * N,                       // mark
        sizeof(int) * kFan6 * N,               // fan6
        sizeof(int) * (kRqWords + 10 * B),      // rq
    };
    size_t off = 0;
    for (int i = 0; i < kLayoutParts; ++i) {
        L->off[i] = off;
        off += align_up(sizes[i]);
    }
    L->total = off;
    return off;
}

Work carve(void* base, const Layout& L) {
    char* b = static_cast<char*>(base);
    Work w;
    w.ctrl = reinterpret_cast<int*>(b + L.off[0]);
    w.mesh = reinterpret_cast<MeshDesc*>(b + L.off[1]);
    w.state = reinterpret_cast<MeshState*>(b + L.off[2]);
    w.wg_prep = reinterpret_cast<WgInfo*>(b + L.off[3]);
    w.glist_prep = reinterpret_cast<int*>(b + L.off[4]);
    w.wg_run = reinterpret_cast<WgInfo*>(b + L.off[5]);
    w.glist_run = reinterpret_cast<int*>(b + L.off[6]);
    w.vo = reinterpret_cast<int*>(b + L.off[7]);
    w.fo3 = reinterpret_cast<int*>(b + L.off[8]);
    w.so = reinterpret_cast<int*>(b + L.off[9]);
    w.level = reinterpret_cast<int*>(b + L.off[10]);
    w.perm = reinterpret_cast<int*>(b + L.off[11]);
    w.iperm = reinterpret_cast<int*>(b + L.off[12]);
    w.offsets = reinterpret_cast<int*>(b + L.off[13]);
    w.rowO = reinterpret_cast<int*>(b + L.off[14]);
    w.wedgeO = reinterpret_cast<int2*>(b + L.off[15]);
    w.cursor = reinterpret_cast<int*>(b + L.off[16]);
    w.fanlen = reinterpret_cast<int*>(b + L.off[17]);
    w.fanO = reinterpret_cast<int*>(b + L.off[18]);
    w.xyz = reinterpret_cast<float4*>(b + L.off[19]);
    w.dist = reinterpret_cast<float*>(b + L.off[20]);
    w.dl = reinterpret_cast<unsigned long long*>(b + L.off[20]);
    w.bits = reinterpret_cast<unsigned*>(b + L.off[22]);
    w.cnt = reinterpret_cast<int*>(b + L.off[23]);
    w.retire = reinterpret_cast<int*>(b + L.off[24]);
    w.scan_tmp = reinterpret_cast<int*>(b + L.off[25]);
    w.bar = reinterpret_cast<unsigned*>(b + L.off[26]);
    w.feat = reinterpret_cast<float4*>(b + L.off[27]);
    w.edge_acc = reinterpret_cast<unsigned long long*>(b + L.off[28]);
    w.lds_mesh = reinterpret_cast<int*>(b + L.off[29]);
    w.fanrow = reinterpret_cast<int2*>(b + L.off[30]);
    w.fan = reinterpret_cast<int*>(b + L.off[31]);
    w.ellO = reinterpret_cast<int*>(b + L.off[32]);
    w.wg_run64 = reinterpret_cast<WgInfo*>(b + L.off[33]);
    w.glist_run64 = reinterpret_cast<int*>(b + L.off[34]);
    w.cvt = reinterpret_cast<double*>(b + L.off[35]);
    w.mark = reinterpret_cast<int*>(b + L.off[36]);
    w.fan6 = reinterpret_cast<int*>(b + L.off[37]);
    w.rq = reinterpret_cast<int*>(b + L.off[38]);
    return w;
}

}  // namespace ptp

// ---- the shared implementation ------------------------------------------
struct Solver {
    std::vector<MeshDesc> mesh;
    std::vector<int> h_vo, h_fo3, h_so;
    Sizes z{};
    ptp_options opt{};
    bool single = false;
    int device = 0, cus = 0, max_prep = 0, max_run = 0, max_run64 = 0, lds_max = 0, big_max = 0;
    // meshes of the one-workgroup BFS (the larger ones, n_big of them, first;
    // each part by decreasing size) and of the grid BFS
    std::vector<int> lds_list, grid_list;
    int n_big = 0;
    ptp_schedule sched{};
    Sched s_prep, s_run, s_run64;
    bool sched64_ready = false;             // s_run64 uploaded for the current prepare
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // prepare begin/end, run begin/end
    float ms_prepare = -1.f;
    bool run_timed = false;
    Layout layout{};
    Work work{};
    hipStream_t stream = nullptr;
    const int32_t* S = nullptr;         // the caller's arrays of the last prepare
    const float* Vp = nullptr;
    const int32_t* Fp = nullptr;
    std::vector<MeshState> hstate;
    std::vector<long long> meas_K, meas_U, meas_rho;   // the last run's K, U and rho per mesh
    bool prepared = false, ran = false;
    bool parents_valid = false;         // the last run computed labels (and parents)
    std::string err;
    int h_ctrl[8];

    ptp_status fail(ptp_status s, const std::string& msg) {
        err = msg;
        return s;
    }
    ptp_status hip_fail(hipError_t e, const char* what) {
        return fail(PTP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }

    ~Solver() {
        for (hipEvent_t& e : ev)
            if (e) (void)hipEventDestroy(e);
    }

    ptp_status init(const ptp_mesh* m, int count, const ptp_options* o, bool one) {
        single = one;
        if (count < 1 || !m) return PTP_EINVAL;
        if (o) {
            opt = *o;
        } else {
            opt.tol = 1e-3f;
            opt.max_iters = 0;
            opt.window = 0;
            opt.want_labels = 0;
            opt.workgroups = 0;
            opt.lds_bfs_max = 0;
            opt.band_rule = PTP_BAND_PAPER;
        }
        if (!(opt.tol > 0.f) || opt.max_iters < 0 || opt.window < 0 || opt.workgroups < 0 ||
            opt.lds_bfs_max < -1 || opt.band_rule < PTP_BAND_PAPER || opt.band_rule > PTP_BAND_JACOBI)
            return PTP_EINVAL;
        long long N = 0, F = 0, Sn = 0, W = 0;
        h_vo.assign(1, 0);
        h_fo3.assign(1, 0);
        h_so.assign(1, 0);
        for (int b = 0; b < count; ++b) {
            const ptp_mesh& d = m[b];
            if (d.n_vertices < 1 || d.n_faces < 0 || d.n_sources < 1 || d.n_sources > d.n_vertices)
                return PTP_EINVAL;
            if (d.v_off < 0 || d.f_off < 0 || d.s_off < 0 || d.out_off < 0) return PTP_EINVAL;
            MeshDesc md;
            md.v_off = (int)N;
            md.f_off = (int)F;
            md.s_off = (int)Sn;
            md.w_off = (int)W;
            md.n = d.n_vertices;
            md.f = d.n_faces;
            md.m = d.n_sources;
            md.pad = 0;
            md.v_in = d.v_off;
            md.f_in = d.f_off;
            md.s_in = d.s_off;
            md.out_off = d.out_off;
            N += d.n_vertices;
            F += d.n_faces;
            Sn += d.n_sources;
            W += (d.n_vertices + 31) / 32;
            if (N > (1ll << 29) || 6 * F >= (1ll << 31) || Sn >= (1ll << 31)) return PTP_EUNSUPPORTED;
            mesh.push_back(md);
            h_vo.push_back((int)N);
            h_fo3.push_back((int)(3 * F));
            h_so.push_back((int)Sn);
        }
        hipError_t e = hipGetDevice(&device);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
        int coop = 0;
        if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device);
        if (e != hipSuccess || !coop || cus < 1) return PTP_EDEVICE;
        for (hipEvent_t& x : ev)
            if (hipEventCreate(&x) != hipSuccess) return PTP_EDEVICE;
        max_prep = max_coop_blocks_bfs(cus);
        const bool rules = opt.band_rule != PTP_BAND_PAPER;
        max_run = max_coop_blocks_run(cus, single, rules);
        max_run64 = max_coop_blocks_run64(cus, rules);
        if (opt.lds_bfs_max >= 0) bfs_one_limits(device, &lds_max, &big_max);
        if (opt.lds_bfs_max > 0) {
            lds_max = std::min(lds_max, opt.lds_bfs_max);
            big_max = std::min(big_max, opt.lds_bfs_max);
        }
        long long lds_words = 0, big_words = 0;
        std::vector<int> small_one;
        for (int b = 0; b < count; ++b) {
            const long long words = (mesh[b].n + 31) / 32;
            if (mesh[b].n <= lds_max) {
                small_one.push_back(b);
                lds_words = std::max(lds_words, words);
            } else if (mesh[b].n <= big_max) {
                lds_list.push_back(b);
                big_words = std::max(big_words, words);
            } else {
                grid_list.push_back(b);
            }
        }
        // largest first: the workgroups of a launch start in index order
        auto by_size = [&](int x, int y) { return mesh[x].n > mesh[y].n; };
        std::stable_sort(lds_list.begin(), lds_list.end(), by_size);
        std::stable_sort(small_one.begin(), small_one.end(), by_size);
        n_big = (int)lds_list.size();
        lds_list.insert(lds_list.end(), small_one.begin(), small_one.end());
        z.lds_words = lds_words;
        z.big_words = big_words;
        z.N = N;
        z.F = F;
        z.S = Sn;
        z.B = count;
        z.W = W;
        z.gmax = std::max(max_prep, std::max(max_run, max_run64));
        sched = default_schedule();
        work_layout(z, &layout);
        return PTP_OK;
    }

    ptp_schedule default_schedule() const {
        ptp_schedule p;
        p.workgroups = std::min(max_run, 4 * cus);
        p.small_limit = 32768;
        p.large_limit = 524288;
        p.medium_group = 8;
        p.large_group = 24;
        p.xcd_pack = 1;
        return p;
    }

    void set_schedule(const ptp_schedule* s) {
        ptp_schedule d = default_schedule();
        if (s) {
            if (s->workgroups > 0) d.workgroups = s->workgroups;
            if (s->small_limit > 0) d.small_limit = s->small_limit;
            if (s->large_limit > 0) d.large_limit = s->large_limit;
            if (s->medium_group > 0) d.medium_group = s->medium_group;
            if (s->large_group > 0) d.large_group = s->large_group;
            if (s->xcd_pack != 0) d.xcd_pack = s->xcd_pack > 0 ? s->xcd_pack : 0;
        }
        sched = d;
    }

    // Single mesh: one group; about one workgroup per 1536 reachable vertices
    // up to 512 (the per-iteration cost is flat from ~n/2048 to ~n/1024
    // workgroups on the icosphere workloads and rises outside).  Up to ~48
    // of them, 32 workgroups placed on one XCD do better (the group then
    // exchanges its data through one L2).
    int single_group(int gmax, long long reach) const {
        if (opt.workgroups > 0) return std::min(opt.workgroups, gmax);
        long long g = reach / 1536;
        g = g <= 48 ? 32 : std::min(512ll, g);
        return (int)std::min<long long>(g, gmax);
    }

    // Relaxation time estimate of each mesh for the scheduler: from the K and
    // U of the last run of the same batch when that run saw the same number
    // of toplesets (the same mesh and sources, most likely), else from rho
    // and n.  The schedule only orders and places the work; results never
    // depend on it.
    CostFn run_cost(const std::vector<long long>& rho) const {
        return [this, &rho](int b, int sz) {
            if (b < (int)meas_rho.size() && meas_rho[b] == rho[b] && meas_K[b] > 0)
                return est_run((double)meas_K[b], (double)meas_U[b], sz);
            return est_run(1.2 * (double)rho[b], 0.2 * (double)mesh[b].n * (double)rho[b], sz);
        };
    }

    // The run launches take their meshes from the queues (Sched::queue).
    hipError_t upload_run(const Sched& s, WgInfo* dwg, int* dq) {
        hipError_t e = hipMemcpyAsync(dwg, s.wg.data(), sizeof(WgInfo) * s.wg.size(), hipMemcpyHostToDevice,
                                      stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dq, s.queue.data(), sizeof(int) * s.queue.size(), hipMemcpyHostToDevice, stream);
        return e;
    }

    hipError_t upload(const Sched& s, WgInfo* dwg, int* dgl) {
        hipError_t e = hipMemcpyAsync(dwg, s.wg.data(), sizeof(WgInfo) * s.wg.size(),
                                      hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dgl, s.glist.data(), sizeof(int) * s.glist.size(), hipMemcpyHostToDevice,
                               stream);
        return e;
    }

    ptp_status prepare(const float* dV, const int32_t* dF, const int32_t* dS, void* dWork,
                       size_t bytes, void* st) {
        prepared = false;
        ran = false;
        parents_valid = false;
        sched64_ready = false;
        ms_prepare = -1.f;
        if (!dV || !dS || (!dF && z.F > 0) || !dWork) return fail(PTP_EINVAL, "null pointer argument");
        if (reinterpret_cast<uintptr_t>(dWork) & 255)
            return fail(PTP_EINVAL, "workspace must be 256-byte aligned");
        if (bytes < layout.total) return fail(PTP_ENOMEM, "workspace smaller than the plan needs");
        stream = static_cast<hipStream_t>(st);
        work = carve(dWork, layout);
        S = dS;
        Vp = dV;
        Fp = dF;
        // the grid BFS takes the meshes too large for one workgroup's LDS.  A
        // level costs a group barrier whatever the group's size, and a level
        // of these meshes holds a few thousand vertices, so the meshes run side
        // by side, one group each (at most one XCD's worth of workgroups),
        // rather than one after another on a few large groups.
        s_prep = Sched{};
        if (!grid_list.empty()) {
            std::vector<MeshDesc> gm;
            std::vector<long long> rho_est;
            for (int b : grid_list) {
                gm.push_back(mesh[b]);
                rho_est.push_back((long long)(2.0 * std::sqrt((double)mesh[b].n)) + 1);
            }
            ptp_schedule ps = sched;
            ps.workgroups = max_prep;
            ps.small_limit = 1;                  // no single-workgroup class
            ps.large_limit = 0x7fffffff;         // every mesh in one class
            ps.medium_group = std::max(1, std::min(32, max_prep / (int)grid_list.size()));
            ps.xcd_pack = 1;
            s_prep = make_schedule(gm, [&](int b, int sz) { return est_time(gm[b].n, rho_est[b], sz); }, ps,
                                   max_prep, grid_list.size() == 1, std::min(cus, max_prep));
            for (size_t x = s_prep.ngroups + 1; x < s_prep.glist.size(); ++x)
                s_prep.glist[x] = grid_list[s_prep.glist[x]];
        }
        hstate.assign(z.B, MeshState{});
        const bool timed = !capturing();
        hipError_t e = timed ? hipEventRecord(ev[0], stream) : hipSuccess;
        if (e == hipSuccess)
            e = hipMemcpyAsync(work.mesh, mesh.data(), sizeof(MeshDesc) * z.B, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(work.vo, h_vo.data(), sizeof(int) * (z.B + 1), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(work.fo3, h_fo3.data(), sizeof(int) * (z.B + 1), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(work.so, h_so.data(), sizeof(int) * (z.B + 1), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(work.state, hstate.data(), sizeof(MeshState) * z.B, hipMemcpyHostToDevice,
                               stream);
        if (e == hipSuccess && s_prep.G > 0) e = upload(s_prep, work.wg_prep, work.glist_prep);
        if (e == hipSuccess && !lds_list.empty())
            e = hipMemcpyAsync(work.lds_mesh, lds_list.data(), sizeof(int) * lds_list.size(),
                               hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "prepare upload");
        e = launch_prepare(work, z, dV, dF, dS, s_prep.G, (int)lds_list.size(), n_big, stream);
        if (e != hipSuccess) return hip_fail(e, "prepare launch");
        if (timed) {
            e = hipEventRecord(ev[1], stream);
            if (e != hipSuccess) return hip_fail(e, "prepare event");
        }
        e = hipMemcpyAsync(h_ctrl, work.ctrl, sizeof(int) * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hstate.data(), work.state, sizeof(MeshState) * z.B, hipMemcpyDeviceToHost,
                               stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "prepare");
        if (timed && hipEventElapsedTime(&ms_prepare, ev[0], ev[1]) != hipSuccess) ms_prepare = -1.f;
        if (h_ctrl[C_ABORT]) return fail(PTP_EDEVICE, "BFS barrier timed out");
        const int stw = h_ctrl[C_STATUS];
        if (stw) {
            std::string msg = "invalid input:";
            if (stw & ST_BAD_FACE) msg += " face index out of range;";
            if (stw & ST_BAD_COORD) msg += " non-finite coordinate;";
            if (stw & ST_BAD_SOURCE) msg += " source index out of range;";
            if (stw & ST_DUP_SOURCE) msg += " duplicate source;";
            return fail(PTP_EINVAL, msg);
        }
        std::vector<long long> rho(z.B);
        long long reach = 0;
        for (int b = 0; b < z.B; ++b) {
            const MeshState& x = hstate[b];
            if (x.rho < 1 || x.reach < mesh[b].m || x.reach > mesh[b].n)
                return fail(PTP_EDEVICE, "BFS produced an inconsistent result");
            rho[b] = x.rho;
            reach += x.reach;
        }
        s_run = make_schedule(mesh, run_cost(rho), sched, max_run, single, single_group(max_run, reach));
        e = upload_run(s_run, work.wg_run, work.glist_run);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "schedule upload");
        prepared = true;
        return PTP_OK;
    }

    bool capturing() const {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        return hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
    }

    // Double-precision schedule: the same work distribution, limited to the
    // workgroups the float64 kernel can keep resident.
    ptp_status ensure_sched64() {
        if (sched64_ready) return PTP_OK;
        std::vector<long long> rho(z.B);
        long long reach = 0;
        for (int b = 0; b < z.B; ++b) {
            rho[b] = hstate[b].rho;
            reach += hstate[b].reach;
        }
        s_run64 = make_schedule(mesh, run_cost(rho), sched, max_run64, single, single_group(max_run64, reach));
        hipError_t e = upload_run(s_run64, work.wg_run64, work.glist_run64);
        if (e != hipSuccess) return hip_fail(e, "schedule upload");
        sched64_ready = true;
        return PTP_OK;
    }

    // dUpper non-null: warm start from that caller-order upper bound
    // (certified, or with certify = false trusted as a supersolution);
    // dDist64 non-null: the float64 run.
    ptp_status run(float* dDist, int32_t* dLabel, void* st, const float* dUpper = nullptr,
                   double* dDist64 = nullptr, bool certify = true) {
        if (!prepared) return fail(PTP_EINVAL, "run before a successful prepare");
        const bool f64 = dDist64 != nullptr;
        if (!dDist && !f64) return fail(PTP_EINVAL, "null distance output");
        const bool labels = opt.want_labels != 0;
        if (labels && dUpper) return fail(PTP_EUNSUPPORTED, "the warm-start entry points return distances only");
        if (f64 && (labels || dUpper))
            return fail(PTP_EUNSUPPORTED, "the float64 run computes distances only, from +inf");
        if (labels && !dLabel) return fail(PTP_EINVAL, "labels wanted: null label output");
        stream = static_cast<hipStream_t>(st);
        if (f64) {
            ptp_status r = ensure_sched64();
            if (r != PTP_OK) return r;
        }
        RunParams rp;
        rp.B = z.B;
        rp.kmax_fixed = opt.max_iters;
        rp.window = opt.window;
        rp.band_rule = opt.band_rule;
        rp.N = z.N;
        rp.tol = opt.tol;
        rp.S = S;
        rp.upper = dUpper;
        rp.certify = certify;
        rp.out_d = dDist;
        rp.out_d64 = dDist64;
        rp.out_l = labels ? dLabel : nullptr;
        rp.Stot = z.S;
        rp.ngroups = f64 ? s_run64.ngroups : s_run.ngroups;
        int nmax = 1;
        for (const MeshDesc& md : mesh) nmax = std::max(nmax, md.n);
        rp.jump_rounds = 1;
        while ((1ll << (rp.jump_rounds - 1)) < nmax) ++rp.jump_rounds;
        run_timed = !capturing();
        hipError_t e = run_timed ? hipEventRecord(ev[2], stream) : hipSuccess;
        if (e == hipSuccess)
            e = launch_run(work, rp, labels, single && !f64, f64, f64 ? s_run64.G : s_run.G, stream);
        if (e == hipSuccess && run_timed) e = hipEventRecord(ev[3], stream);
        if (e != hipSuccess) return hip_fail(e, "run launch");
        ran = true;
        parents_valid = labels;
        return PTP_OK;
    }

    // The parents behind the labels of the last run (caller order).
    ptp_status get_parents(int32_t* dParent, void* st) {
        if (!dParent) return fail(PTP_EINVAL, "null parent output");
        if (!parents_valid) return fail(PTP_EINVAL, "parents come with the labels of a labelled run");
        stream = static_cast<hipStream_t>(st);
        const hipError_t e = launch_parents_out(work, z.B, z.N, dParent, stream);
        if (e != hipSuccess) return hip_fail(e, "parents launch");
        return PTP_OK;
    }

    // Farthest point sampling (Sec. 5.3) on a single mesh: S[0, n0) are the
    // caller's sources; S[n0, m) receive the samples.  Every step is enqueued
    // without a host round trip: run, farthest vertex, BFS + reorder.
    ptp_status fps(const float* dV, const int32_t* dF, int32_t* dS, int n0, void* dWork, size_t bytes,
                   bool warm, float* dDist, float* dRadius, int64_t* dSteps, void* st) {
        if (!single || z.B != 1) return fail(PTP_EINVAL, "sampling runs on a single-mesh plan");
        if (opt.want_labels) return fail(PTP_EUNSUPPORTED, "sampling computes distances only");
        const int mt = mesh[0].m;
        if (n0 < 1 || n0 > mt) return fail(PTP_EINVAL, "n_initial must be in [1, n_sources]");
        if (!dDist) return fail(PTP_EINVAL, "null distance output");
        // validate and prepare with the first n0 sources
        mesh[0].m = n0;
        h_so[1] = n0;
        const long long zs = z.S;
        z.S = n0;
        ptp_status r = prepare(dV, dF, dS, dWork, bytes, st);
        mesh[0].m = mt;
        h_so[1] = mt;
        z.S = zs;
        if (r != PTP_OK) return r;
        const int n = mesh[0].n;
        hipError_t e = hipSuccess;
        for (int slot = n0;; ++slot) {
            r = run(dDist, nullptr, st, warm && slot > n0 ? dDist : nullptr, nullptr, false);
            if (r != PTP_OK) return r;
            int64_t* step = dSteps ? dSteps + 2 * (size_t)(slot - n0) : nullptr;
            if (slot == mt) {
                e = launch_fps_pick(work, dDist, n, dS, -1, nullptr, reinterpret_cast<long long*>(step), stream);
                break;
            }
            e = launch_fps_pick(work, dDist, n, dS, slot, dRadius ? dRadius + (slot - n0) : nullptr,
                                reinterpret_cast<long long*>(step), stream);
            if (e == hipSuccess)
                e = launch_prepare_bfs(work, z, dV, dS, s_prep.G, (int)lds_list.size(), n_big, stream);
            if (e != hipSuccess) break;
        }
        if (e == hipSuccess) e = hipMemcpyAsync(h_ctrl, work.ctrl, sizeof(int) * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "sampling");
        if (h_ctrl[C_STATUS] & ST_FPS_EMPTY)
            return fail(PTP_EINVAL, "fewer reachable vertices than samples requested");
        if (h_ctrl[C_STATUS]) return fail(PTP_EINVAL, "invalid input during sampling");
        return stats(nullptr, nullptr);
    }

    // One Lloyd step on the labels of the last run (caller order), over the
    // mesh and sources of the last prepare (validated there).
    ptp_status lloyd_step(const int32_t* dLabel, int32_t* dSout, double* dCentroid, void* st) {
        if (!single || z.B != 1) return fail(PTP_EINVAL, "Lloyd steps run on a single-mesh plan");
        if (!prepared) return fail(PTP_EINVAL, "Lloyd step before a successful prepare");
        if (!dLabel || !dSout) return fail(PTP_EINVAL, "null pointer argument");
        if (dSout == S) return fail(PTP_EINVAL, "the new generators may not overwrite the sources");
        stream = static_cast<hipStream_t>(st);
        const int m = mesh[0].m;
        double* cen = dCentroid ? dCentroid : work.cvt + (size_t)z.S * kCvtChunks * 6;
        hipError_t e = launch_lloyd(work, Vp, Fp, mesh[0].n, mesh[0].f, dLabel, S, m, dSout, cen, stream);
        if (e != hipSuccess) return hip_fail(e, "Lloyd launch");
        return PTP_OK;
    }

    ptp_status warm_features(float* dX, float* dScale, void* st) {
        if (!prepared) return fail(PTP_EINVAL, "features before a successful prepare");
        if (!dX || !dScale) return fail(PTP_EINVAL, "null feature output");
        stream = static_cast<hipStream_t>(st);
        hipError_t e = launch_features(work, z, stream);
        if (e == hipSuccess) e = launch_export_features(work, z, dX, dScale, stream);
        if (e != hipSuccess) return hip_fail(e, "features launch");
        return PTP_OK;
    }

    ptp_status warm_predict(const float* dParams, float inflate, float* dUpper, void* st) {
        if (!prepared) return fail(PTP_EINVAL, "predict before a successful prepare");
        if (!dParams || !dUpper) return fail(PTP_EINVAL, "null parameters or output");
        if (!(inflate >= 1.f) || !std::isfinite(inflate)) return fail(PTP_EINVAL, "inflate must be >= 1");
        stream = static_cast<hipStream_t>(st);
        hipError_t e = launch_features(work, z, stream);
        if (e == hipSuccess) e = launch_predict(work, z, dParams, inflate, dUpper, stream);
        if (e != hipSuccess) return hip_fail(e, "predict launch");
        return PTP_OK;
    }

    ptp_status stats(ptp_stats* out, int32_t* status) {
        if (!ran) return fail(PTP_EINVAL, "no run to report");
        hipError_t e = hipMemcpyAsync(h_ctrl, work.ctrl, sizeof(int) * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hstate.data(), work.state, sizeof(MeshState) * z.B, hipMemcpyDeviceToHost,
                               stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "stats");
        float ms_run = -1.f;
        if (run_timed && hipEventElapsedTime(&ms_run, ev[2], ev[3]) != hipSuccess) ms_run = -1.f;
        meas_K.assign(z.B, 0);
        meas_U.assign(z.B, 0);
        meas_rho.assign(z.B, -1);
        for (int b = 0; b < z.B; ++b)
            if (!h_ctrl[C_ABORT] && !hstate[b].status && !hstate[b].runstat) {
                meas_K[b] = hstate[b].iters;
                meas_U[b] = hstate[b].updates;
                meas_rho[b] = hstate[b].rho;
            }
        long long t0 = 0;
        for (int b = 0; b < z.B; ++b)
            if (hstate[b].t_begin && (!t0 || hstate[b].t_begin < t0)) t0 = hstate[b].t_begin;
        ptp_status agg = PTP_OK;
        for (int b = 0; b < z.B; ++b) {
            const MeshState& x = hstate[b];
            ptp_status sb = PTP_OK;
            if (x.status) sb = PTP_EINVAL;
            else if (h_ctrl[C_ABORT]) sb = PTP_EDEVICE;
            else if (x.runstat) sb = PTP_ENOCONV;
            if (status) status[b] = sb;
            if (out) {
                out[b].iterations = x.iters;
                out[b].n_toplesets = x.rho;
                out[b].reachable = x.reach;
                out[b].workgroups = x.wgs > 0 ? x.wgs : s_run.gsize_of[b];
                out[b].vertex_updates = x.updates;
                out[b].certify_rounds = x.cert_rounds;
                out[b].certify_rejected = x.cert_rejected;
                out[b].ms_prepare = ms_prepare;
                out[b].ms_run = ms_run;
                // device wall clock at 100 MHz
                out[b].ms_mesh_begin = x.t_begin ? (float)((x.t_begin - t0) * 1e-5) : -1.f;
                out[b].ms_mesh_end = x.t_end ? (float)((x.t_end - t0) * 1e-5) : -1.f;
                out[b].evaluated_updates = (int64_t)x.evaluated;
            }
            if (agg == PTP_OK && sb != PTP_OK) agg = sb;
        }
        if (h_ctrl[C_ABORT]) return fail(PTP_EDEVICE, "relaxation barrier timed out");
        if (agg == PTP_ENOCONV) return fail(PTP_ENOCONV, "iteration cap reached");
        return agg;
    }

    ptp_status autotune(const ptp_schedule* cand, int n, float* dDist, int32_t* dLabel, float* hMs,
                        int32_t* best, void* st) {
        if (!prepared) return fail(PTP_EINVAL, "autotune before a successful prepare");
        if (!cand || n < 1) return fail(PTP_EINVAL, "no candidate schedules");
        stream = static_cast<hipStream_t>(st);
        std::vector<long long> rho(z.B);
        long long reach = 0;
        for (int b = 0; b < z.B; ++b) {
            rho[b] = hstate[b].rho;
            reach += hstate[b].reach;
        }
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return fail(PTP_EDEVICE, "event");
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(PTP_EDEVICE, "event");
        }
        const ptp_schedule keep = sched;
        int bi = -1;
        float bms = 0.f;
        ptp_status rc = PTP_OK;
        for (int c = 0; c < n && rc == PTP_OK; ++c) {
            set_schedule(&cand[c]);
            s_run = make_schedule(mesh, run_cost(rho), sched, max_run, single, single_group(max_run, reach));
            hipError_t e = upload_run(s_run, work.wg_run, work.glist_run);
            if (e != hipSuccess) {
                rc = hip_fail(e, "schedule upload");
                break;
            }
            rc = run(dDist, dLabel, st);                  // warm-up
            if (rc != PTP_OK) break;
            e = hipEventRecord(e0, stream);
            if (e == hipSuccess) rc = run(dDist, dLabel, st);
            if (e == hipSuccess && rc == PTP_OK) e = hipEventRecord(e1, stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = hip_fail(e, "autotune timing");
                break;
            }
            ptp_status sr = stats(nullptr, nullptr);
            if (sr == PTP_EDEVICE) {
                rc = sr;
                break;
            }
            if (hMs) hMs[c] = ms;
            if (bi < 0 || ms < bms) {
                bi = c;
                bms = ms;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != PTP_OK) {
            sched = keep;
            return rc;
        }
        set_schedule(&cand[bi]);
        s_run = make_schedule(mesh, run_cost(rho), sched, max_run, single, single_group(max_run, reach));
        hipError_t e = upload_run(s_run, work.wg_run, work.glist_run);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "schedule upload");
        if (best) *best = bi;
        return PTP_OK;
    }
};

struct ptp_plan {
    Solver s;
};
struct ptp_batch {
    Solver s;
};

// ---- fixed scratch for callers that cannot allocate ---------------------
// ptp_solve_noalloc carves its workspace from this array instead of a
// caller buffer.  Each device holds its own copy from the moment the library
// is loaded until the process ends.  In host code `scratch` names a host-side
// stand-in, not the device address: the address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on the first
// call made with that device current).
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

extern "C" {

const char* ptp_version(void) { return "ptp-mi355x 0.4 (gfx950)"; }

// ---- one mesh ------------------------------------------------------------
ptp_status ptp_plan_create(ptp_plan** out, int32_t n, int32_t f, int32_t m, const ptp_options* opt) {
    if (!out) return PTP_EINVAL;
    *out = nullptr;
    if (n < 1 || f < 0 || m < 1 || m > n) return PTP_EINVAL;
    if (n > (1 << 29) || (long long)f * 3 >= (1ll << 31)) return PTP_EUNSUPPORTED;
    if (opt && (!(opt->tol > 0.f) || opt->max_iters < 0 || opt->window < 0 || opt->workgroups < 0 ||
                opt->band_rule < PTP_BAND_PAPER || opt->band_rule > PTP_BAND_JACOBI))
        return PTP_EINVAL;
    ptp_plan* p = new (std::nothrow) ptp_plan();
    if (!p) return PTP_ENOMEM;
    ptp_mesh d;
    d.v_off = d.f_off = d.s_off = d.out_off = 0;
    d.n_vertices = n;
    d.n_faces = f;
    d.n_sources = m;
    d.reserved = 0;
    ptp_status s = p->s.init(&d, 1, opt, true);
    if (s != PTP_OK) {
        delete p;
        return s;
    }
    *out = p;
    return PTP_OK;
}

ptp_status ptp_workspace_bytes(const ptp_plan* p, size_t* bytes) {
    if (!p || !bytes) return PTP_EINVAL;
    *bytes = p->s.layout.total;
    return PTP_OK;
}

ptp_status ptp_prepare(ptp_plan* p, const float* dV, const int32_t* dF, const int32_t* dS,
                       void* dWork, size_t work_bytes, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.prepare(dV, dF, dS, dWork, work_bytes, stream);
}

ptp_status ptp_run(ptp_plan* p, float* dDist, int32_t* dLabel, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.run(dDist, dLabel, stream);
}

ptp_status ptp_get_stats(ptp_plan* p, ptp_stats* st) {
    if (!p) return PTP_EINVAL;
    return p->s.stats(st, nullptr);
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

ptp_status ptp_solve_noalloc(ptp_plan* p, const float* dV, const int32_t* dF, const int32_t* dS, float* dDist,
                             int32_t* dLabel, ptp_stats* stats, void* stream) {
    if (!p) return PTP_EINVAL;
    Solver& s = p->s;
    if (s.layout.total > kScratchBytes)
        return s.fail(PTP_ENOMEM, "the plan needs " + std::to_string(s.layout.total) +
                                      " bytes of workspace; the fixed scratch holds " +
                                      std::to_string(kScratchBytes));
    void* work = nullptr;
    const hipError_t e = scratch_address(&work);
    if (e != hipSuccess) return s.hip_fail(e, "scratch address");
    return ptp_solve(p, dV, dF, dS, work, kScratchBytes, dDist, dLabel, stats, stream);
}

size_t ptp_noalloc_scratch_bytes(void) { return kScratchBytes; }

ptp_status ptp_run_f64(ptp_plan* p, double* dDist, void* stream) {
    if (!p) return PTP_EINVAL;
    if (!dDist) return p->s.fail(PTP_EINVAL, "null distance output");
    return p->s.run(nullptr, nullptr, stream, nullptr, dDist);
}

ptp_status ptp_fps(ptp_plan* p, const float* dV, const int32_t* dF, int32_t* dS, int32_t n_initial,
                   void* dWork, size_t work_bytes, int32_t warm, float* dDist, float* dRadius, int64_t* dSteps,
                   void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.fps(dV, dF, dS, n_initial, dWork, work_bytes, warm != 0, dDist, dRadius, dSteps, stream);
}

ptp_status ptp_lloyd_step(ptp_plan* p, const int32_t* dLabel, int32_t* dSout, double* dCentroid, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.lloyd_step(dLabel, dSout, dCentroid, stream);
}

ptp_status ptp_get_parents(ptp_plan* p, int32_t* dParent, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.get_parents(dParent, stream);
}

ptp_status ptp_get_order(ptp_plan* p, int32_t* dPerm, int32_t* dOffsets, void* stream) {
    if (!p) return PTP_EINVAL;
    Solver& s = p->s;
    if (!s.prepared) return s.fail(PTP_EINVAL, "no prepared mesh");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (dPerm)
        e = hipMemcpyAsync(dPerm, s.work.perm, sizeof(int) * (size_t)s.z.N, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && dOffsets)
        e = hipMemcpyAsync(dOffsets, s.work.offsets, sizeof(int) * ((size_t)s.hstate[0].rho + 1),
                           hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return s.hip_fail(e, "get_order");
    return PTP_OK;
}

ptp_status ptp_get_schedule(ptp_plan* p, int32_t* hRetire) {
    if (!p || !hRetire) return PTP_EINVAL;
    Solver& s = p->s;
    if (!s.ran) return s.fail(PTP_EINVAL, "no run to report");
    hipError_t e = hipMemcpyAsync(hRetire, s.work.retire, sizeof(int) * (size_t)s.hstate[0].rho,
                                  hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    if (e != hipSuccess) return s.hip_fail(e, "get_schedule");
    return PTP_OK;
}

int32_t ptp_n_toplesets(const ptp_plan* p) {
    return p && p->s.prepared ? p->s.hstate[0].rho : -1;
}

ptp_status ptp_warm_features(ptp_plan* p, float* dX, float* dScale, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.warm_features(dX, dScale, stream);
}

ptp_status ptp_warm_predict(ptp_plan* p, const float* dParams, float inflate, float* dUpper, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.warm_predict(dParams, inflate, dUpper, stream);
}

ptp_status ptp_run_warm(ptp_plan* p, const float* dUpper, float* dDist, void* stream) {
    if (!p) return PTP_EINVAL;
    if (!dUpper) return p->s.fail(PTP_EINVAL, "null upper bound");
    return p->s.run(dDist, nullptr, stream, dUpper);
}

ptp_status ptp_set_window(ptp_plan* p, int32_t window) {
    if (!p) return PTP_EINVAL;
    if (window < 0) return p->s.fail(PTP_EINVAL, "negative window");
    p->s.opt.window = window;
    return PTP_OK;
}

const char* ptp_last_error(const ptp_plan* p) { return p ? p->s.err.c_str() : "null plan"; }

void ptp_plan_destroy(ptp_plan* p) { delete p; }

// ---- batches -------------------------------------------------------------
ptp_status ptp_batch_create(ptp_batch** out, const ptp_mesh* meshes, int32_t count,
                            const ptp_options* opt) {
    if (!out) return PTP_EINVAL;
    *out = nullptr;
    if (!meshes || count < 1) return PTP_EINVAL;
    ptp_batch* p = new (std::nothrow) ptp_batch();
    if (!p) return PTP_ENOMEM;
    ptp_status s = p->s.init(meshes, count, opt, false);
    if (s != PTP_OK) {
        delete p;
        return s;
    }
    *out = p;
    return PTP_OK;
}

ptp_status ptp_batch_workspace_bytes(const ptp_batch* p, size_t* bytes) {
    if (!p || !bytes) return PTP_EINVAL;
    *bytes = p->s.layout.total;
    return PTP_OK;
}

ptp_status ptp_batch_prepare(ptp_batch* p, const float* dV, const int32_t* dF, const int32_t* dS,
                             void* dWork, size_t work_bytes, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.prepare(dV, dF, dS, dWork, work_bytes, stream);
}

ptp_status ptp_batch_run(ptp_batch* p, float* dDist, int32_t* dLabel, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.run(dDist, dLabel, stream);
}

ptp_status ptp_batch_run_f64(ptp_batch* p, double* dDist, void* stream) {
    if (!p) return PTP_EINVAL;
    if (!dDist) return p->s.fail(PTP_EINVAL, "null distance output");
    return p->s.run(nullptr, nullptr, stream, nullptr, dDist);
}

ptp_status ptp_batch_get_stats(ptp_batch* p, ptp_stats* hStats, int32_t* hStatus) {
    if (!p) return PTP_EINVAL;
    Solver& s = p->s;
    if (!s.ran) {   // after a failed prepare: report which meshes were invalid
        if (hStatus)
            for (int b = 0; b < s.z.B; ++b)
                hStatus[b] = (b < (int)s.hstate.size() && s.hstate[b].status) ? PTP_EINVAL : PTP_OK;
        return s.fail(PTP_EINVAL, "no run to report");
    }
    return s.stats(hStats, hStatus);
}

ptp_status ptp_batch_get_parents(ptp_batch* p, int32_t* dParent, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.get_parents(dParent, stream);
}

ptp_status ptp_batch_set_window(ptp_batch* p, int32_t window) {
    if (!p) return PTP_EINVAL;
    if (window < 0) return p->s.fail(PTP_EINVAL, "negative window");
    p->s.opt.window = window;
    return PTP_OK;
}

ptp_status ptp_batch_set_schedule(ptp_batch* p, const ptp_schedule* sch) {
    if (!p) return PTP_EINVAL;
    if (sch && (sch->workgroups < 0 || sch->small_limit < 0 || sch->large_limit < 0 ||
                sch->medium_group < 0 || sch->large_group < 0))
        return p->s.fail(PTP_EINVAL, "negative schedule field");
    p->s.set_schedule(sch);
    return PTP_OK;
}

ptp_status ptp_batch_get_schedule(const ptp_batch* p, ptp_schedule* sch) {
    if (!p || !sch) return PTP_EINVAL;
    *sch = p->s.sched;
    return PTP_OK;
}

ptp_status ptp_batch_autotune(ptp_batch* p, const ptp_schedule* candidates, int32_t n, float* dDist,
                              int32_t* dLabel, float* hMs, int32_t* best, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.autotune(candidates, n, dDist, dLabel, hMs, best, stream);
}

ptp_status ptp_batch_warm_features(ptp_batch* p, float* dX, float* dScale, void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.warm_features(dX, dScale, stream);
}

ptp_status ptp_batch_warm_predict(ptp_batch* p, const float* dParams, float inflate, float* dUpper,
                                  void* stream) {
    if (!p) return PTP_EINVAL;
    return p->s.warm_predict(dParams, inflate, dUpper, stream);
}

ptp_status ptp_batch_run_warm(ptp_batch* p, const float* dUpper, float* dDist, void* stream) {
    if (!p) return PTP_EINVAL;
    if (!dUpper) return p->s.fail(PTP_EINVAL, "null upper bound");
    return p->s.run(dDist, nullptr, stream, dUpper);
}

const char* ptp_batch_last_error(const ptp_batch* p) { return p ? p->s.err.c_str() : "null batch"; }

void ptp_batch_destroy(ptp_batch* p) { delete p; }

// ---- the warm-start network ----------------------------------------------
int32_t ptp_mlp_params(void) { return kParams; }

size_t ptp_mlp_scratch_bytes(void) { return mlp_scratch_bytes(); }

ptp_status ptp_mlp_apply(const float* dParams, const float* dX, const float* dScale, int64_t n, float* dOut,
                         void* stream) {
    if (!dParams || n < 0 || (n > 0 && (!dX || !dScale || !dOut))) return PTP_EINVAL;
    if (n == 0) return PTP_OK;
    return launch_mlp_apply(dParams, dX, dScale, n, dOut, static_cast<hipStream_t>(stream)) == hipSuccess
               ? PTP_OK
               : PTP_EDEVICE;
}

ptp_status ptp_mlp_grad(const float* dParams, const float* dX, const float* dScale, const float* dTarget,
                        int64_t n, void* dScratch, size_t scratch_bytes, float* dGrad, float* dLoss,
                        void* stream) {
    if (!dParams || !dX || !dScale || !dTarget || !dScratch || !dGrad || n < 1) return PTP_EINVAL;
    if (reinterpret_cast<uintptr_t>(dScratch) & 15) return PTP_EINVAL;
    if (scratch_bytes < mlp_scratch_bytes()) return PTP_ENOMEM;
    return launch_mlp_grad(dParams, dX, dScale, dTarget, n, static_cast<float*>(dScratch), dGrad, dLoss,
                           static_cast<hipStream_t>(stream)) == hipSuccess
               ? PTP_OK
               : PTP_EDEVICE;
}

ptp_status ptp_adam_step(float* dParams, const float* dGrad, float* dM, float* dV, int32_t t, float lr,
                         float beta1, float beta2, float eps, void* stream) {
    if (!dParams || !dGrad || !dM || !dV || t < 1) return PTP_EINVAL;
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return PTP_EINVAL;
    return launch_adam(dParams, dGrad, dM, dV, t, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? PTP_OK
               : PTP_EDEVICE;
}

}  // extern "C"
