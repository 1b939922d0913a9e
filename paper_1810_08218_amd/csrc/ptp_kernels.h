// Internal interface between the host API and the kernel sources.
//
// Every solve is a batch: B meshes concatenated in the caller's arrays
// (one mesh is a batch of one).  Vertex, face and source ids inside each
// mesh are local; the library works on the concatenation, in which mesh b
// owns the positions [v_off_b, v_off_b + n_b).  The persistent kernels run
// "groups" of consecutive workgroups; each group takes its meshes one after
// the other, with a barrier of its own.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ptp {

struct MeshDesc {          // per mesh, host and device
    int v_off, f_off, s_off, w_off;     // internal prefixes: vertices, faces, sources, bitmap words
    int n, f, m, pad;                   // sizes
    long long v_in, f_in, s_in;         // first row / entry in the caller's V, F, S
    long long out_off;                  // first entry in the caller's outputs
};

struct MeshState {         // per mesh, written by the kernels
    int status;            // StatusBits of the mesh
    int rho, reach;        // toplesets, reachable vertices
    int iters, runstat;    // K, 1 = cap reached
    float mean_edge;       // mean edge length (warm-start features)
    long long updates;     // U
    int cert_rounds;       // warm start: certification sweeps
    int cert_rejected;     // warm start: bounds withdrawn by the certification
};

struct WgInfo {            // per workgroup of a persistent launch
    int group, rank, gsize, first;
};

// Device workspace, carved from the caller's buffer.
struct Work {
    int* ctrl;          // C_WORDS control words (batch-wide)
    MeshDesc* mesh;     // [B]
    MeshState* state;   // [B]
    WgInfo* wg_prep;    // [gmax]  group layout of the BFS launch
    int* glist_prep;    // [gmax + 1 + B] per-group mesh lists (CSR: starts then ids)
    WgInfo* wg_run;     // [gmax]  group layout of the relaxation launch
    int* glist_run;     // [gmax + 1 + B]
    int* vo;            // [B + 1] internal vertex prefix (mesh of a position / vertex)
    int* fo3;           // [B + 1] 3 * internal face prefix (mesh of a face corner)
    int* so;            // [B + 1] internal source prefix (mesh of a source)
    int* level;         // [N]     hop distance by global vertex id (-1 unreachable)
    int* perm;          // [N]     position -> global vertex id
    int* iperm;         // [N]     global vertex id -> position
    int* offsets;       // [N + B] topleset starts, mesh b at v_off_b + b
    int* rowO;          // [N + 1] incidence CSR over global vertex ids
    int2* wedgeO;       // [3F]    opposite edge of each incident triangle, global ids
    int* cursor;        // [N]     fill cursors
    int* rowN;          // [N + 1] incidence CSR over positions
    int2* wedge;        // [3F]    opposite edge, positions
    float4* xyz;        // [N]     coordinates by position (w unused)
    float* dist;        // [2N]    Jacobi double buffer
    unsigned long long* dl;   // [2N] (distance, label) double buffer of the labelled run
    unsigned* bits;     // [2 * W] frontier bitmaps, mesh b at 2 * w_off_b
    int* cnt;           // [4 * gmax] per-workgroup chunk counts
    int* retire;        // [N]     last iteration that updated each topleset, mesh b at v_off_b
    int* scan_tmp;      // block sums of the scans
    unsigned* bar;      // [32 * 2 * gmax] barrier lines: two banks of one line per workgroup
    float4* feat;       // [N]     warm-start network inputs and scale per position
    unsigned long long* edge_acc;   // [2B] fixed-point edge-length sums, then maxima
    int* lds_mesh;      // [B]     meshes of the one-workgroup BFS
    int* fanrow;        // [N + 1] fan CSR over positions
    int* fan;           // [6F]    fans of the incident triangles, positions and flags
    int* ellO;          // [kEll * N] distinct neighbours by global vertex id (BFS)
};

constexpr int kLayoutParts = 33;

// Neighbour rows of the BFS: the distinct neighbours of a vertex in one
// 32-byte row, padded with -1; a vertex with more keeps kEllMore in its last
// entry and is expanded from its incidence instead.
constexpr int kEll = 8;
constexpr int kEllMore = -2;

// Fan of a position: its incident triangles as chains of neighbours.  Wedges
// (a, b) and (b, c) of triangles adjacent around the vertex share b, so a
// chain a, b, c, ... names every neighbour once and the triangles are its
// consecutive pairs, each in its wedge's own orientation.  An entry is a
// position with flags: kFanStart opens a chain (no triangle with the entry
// before it); kFanClosed on entry 0 of a fan that is one closed chain stands
// for the triangle (last entry, entry 0).  A fan has at most 2 * degree
// entries (every wedge a chain of its own).
constexpr int kFanStart = (int)0x80000000u;
constexpr int kFanClosed = 1 << 30;
constexpr int kFanId = kFanClosed - 1;
constexpr int kFanChainMax = 16;     // above this degree every wedge is a chain of its own

struct Sizes {
    long long N, F, S;      // internal totals over the batch
    int B;                  // meshes
    long long W;            // bitmap words (sum over meshes)
    long long lds_words;    // largest bitmap (words) among the one-workgroup BFS meshes
    int gmax;               // largest persistent grid
};

struct Layout {
    size_t off[kLayoutParts];
    size_t total;
};

size_t work_layout(const Sizes& z, Layout* L);
Work carve(void* base, const Layout& L);

// prepare: every kernel after validation is gated on the batch status word
// n_lds meshes (ids in w.lds_mesh) take the one-workgroup LDS BFS, the
// others the persistent grid BFS on g_prep workgroups (0: none).
hipError_t launch_prepare(const Work& w, const Sizes& z, const float* V, const int* F,
                          const int* S, int g_prep, int n_lds, hipStream_t st);
size_t bfs_lds_bytes(long long words);
int bfs_lds_max_vertices(int device);

// zero the barrier lines (two banks of one per workgroup) of a launch
void launch_barrier_reset(const Work& w, int lines, hipStream_t st);

struct RunParams {
    int B, kmax_fixed, window;   // kmax_fixed 0: 4 rho + 16 per mesh
    long long N;
    float tol;
    const int* S;
    const float* upper;          // warm start: caller-order upper bound, or null
    float* out_d;
    int* out_l;
};

// cache: use the register-caching relaxation (single meshes)
hipError_t launch_run(const Work& w, const RunParams& p, bool labels, bool cache, int g_run,
                      hipStream_t st);

// learned warm start
hipError_t launch_features(const Work& w, const Sizes& z, hipStream_t st);
hipError_t launch_export_features(const Work& w, const Sizes& z, float* X, float* scale, hipStream_t st);
hipError_t launch_predict(const Work& w, const Sizes& z, const float* params, float inflate, float* upper,
                          hipStream_t st);
hipError_t launch_mlp_apply(const float* params, const float* X, const float* S, long long n, float* out,
                            hipStream_t st);
hipError_t launch_mlp_grad(const float* params, const float* X, const float* S, const float* D, long long n,
                           float* scratch, float* grad, float* loss, hipStream_t st);
hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int t, float lr, float b1,
                       float b2, float eps, hipStream_t st);
size_t mlp_scratch_bytes();

int max_coop_blocks_bfs(int cus);
int max_coop_blocks_run(int cus, bool labels, bool cache);

}  // namespace ptp
