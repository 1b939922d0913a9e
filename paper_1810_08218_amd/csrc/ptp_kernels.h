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
    long long t_begin;     // device wall clock (100 MHz ticks) when the group
    long long t_end;       //   started / finished this mesh's iteration
    int wgs;               // workgroups of the group that ran it
    int pad2;
    unsigned long long evaluated;   // band positions whose triangles were evaluated
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
    int* glist_prep;    // [gmax + 8 + B] per-group mesh lists (CSR: starts then ids)
    WgInfo* wg_run;     // [gmax]  group layout of the relaxation launch
    int* glist_run;     // [gmax + 8 + B] mesh queues of the relaxation launch (Sched::queue)
    int* vo;            // [B + 1] internal vertex prefix (mesh of a position / vertex)
    int* fo3;           // [B + 1] 3 * internal face prefix (mesh of a face corner)
    int* so;            // [B + 1] internal source prefix (mesh of a source)
    int* level;         // [N]     hop distance by global vertex id (-1 unreachable)
    int* perm;          // [N]     position -> global vertex id
    int* iperm;         // [N]     global vertex id -> position
    int* offsets;       // [N + B] topleset starts, mesh b at v_off_b + b
    int* rowO;          // [N + 1] incidence CSR over global vertex ids
    int2* wedgeO;       // [3F]    opposite edge of each incident triangle, global ids
    int* cursor;        // [N]     fill cursors; after a labelled run the parents (positions)
    int* fanlen;        // [N + 1] fan length of each vertex (global ids)
    int* fanO;          // [6F + 2] fans by global vertex id, vertex v at 2 * rowO[v]
    float4* xyz;        // [N]     coordinates by position (w unused)
    float* dist;        // [2N]    Jacobi double buffer (plain and warm runs)
    unsigned long long* dl;   // [2N] the same memory as 8-byte entries: (distance, label)
                              // pairs of the labelled run, doubles of the float64 run
    unsigned* bits;     // [2 * W] frontier bitmaps, mesh b at 2 * w_off_b
    int* cnt;           // [4 * gmax] per-workgroup chunk counts
    int* retire;        // [N]     last iteration that updated each topleset, mesh b at v_off_b
    int* scan_tmp;      // block sums of the scans
    unsigned* bar;      // [32 * 2 * gmax] barrier lines: two banks of one line per workgroup
    float4* feat;       // [N]     warm-start network inputs and scale per position
    unsigned long long* edge_acc;   // [2B] fixed-point edge-length sums, then maxima
    int* lds_mesh;      // [B]     meshes of the one-workgroup BFS
    int2* fanrow;       // [N]     (start, end) in fan of each position whose fan is longer than kFan6
    int* fan;           // [6F]    those fans' entries, positions and flags, at twice the vertex's incidence offset
    int* ellO;          // [kEll * N] distinct neighbours by global vertex id (BFS)
    WgInfo* wg_run64;   // [gmax]  group layout of the double-precision relaxation
    int* glist_run64;   // [gmax + 8 + B]
    double* cvt;        // [S * kCvtChunks * 6] partial cell sums of the Lloyd step
    int* mark;          // [N]     per position: the last iteration + 1 in which a neighbour changed
    int* fan6;          // [6N]    per position its first kFan6 fan entries in a fixed-size record
    int* rq;            // [kRqWords + 10B] queues of the reorder inside the one-workgroup BFS
};

constexpr int kLayoutParts = 39;

// The reorder of a batch inside its one-workgroup BFS launch.  A workgroup
// that has finished its mesh's BFS publishes the mesh in the queue of the XCD
// it runs on (the positions were written through that XCD's L2), or, for the
// last meshes to finish, in a queue shared by all XCDs after writing its L2
// back; it then reorders chunks of published meshes.  rq: kRqWords control
// words (RqWord; RQ_SLOTS + x: slots taken in the queue of XCD x), then eight
// queues of B slots (mesh + 1; 0 until published), the shared queue of B
// slots, then per mesh the number of its chunks claimed.  Zeroed before the
// launch.
constexpr int kRqWords = 16;
enum RqWord : int { RQ_STARTED = 0, RQ_FINISHED = 1, RQ_FINISHING = 2, RQ_SHARED = 3, RQ_SLOTS = 8 };

// Lloyd step: every cell's sums are split over this many chunks of the
// faces (or vertices), each reduced in a fixed order.
constexpr int kCvtChunks = 64;

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
constexpr int kFanId = (1 << 29) - 1;    // positions stay below 2^29

// The same fans as records of kFan6 entries per position (fan6), read by
// position without the fan row: entries past the fan's length carry kFan6Pad
// and entry 0's id; a fan longer than kFan6 has kFan6Pad on its entry 0 and
// continues in the row form; an empty fan is the position itself without
// kFanStart (every non-empty fan opens with kFanStart).
constexpr int kFan6 = 6;
constexpr int kFan6Pad = 1 << 29;
constexpr int kFanChainMax = 16;     // above this degree every wedge is a chain of its own

struct Sizes {
    long long N, F, S;      // internal totals over the batch
    int B;                  // meshes
    long long W;            // bitmap words (sum over meshes)
    long long lds_words;    // largest bitmap (words) among the meshes of the one-workgroup LDS BFS
    long long big_words;    // the same among the larger one-workgroup BFS meshes (frontier in memory)
    int gmax;               // largest persistent grid
};

struct Layout {
    size_t off[kLayoutParts];
    size_t total;
};

size_t work_layout(const Sizes& z, Layout* L);
Work carve(void* base, const Layout& L);

// prepare: every kernel after validation is gated on the batch status word
// n_one meshes (ids in w.lds_mesh, the n_big larger ones first) take the
// one-workgroup BFS, the others the persistent grid BFS on g_prep
// workgroups (0: none).
hipError_t launch_prepare(const Work& w, const Sizes& z, const float* V, const int* F,
                          const int* S, int g_prep, int n_one, int n_big, hipStream_t st);
size_t bfs_one_bytes(long long lds_words, long long big_words);
void bfs_one_limits(int device, int* lds_max, int* big_max);

// zero the barrier lines (two banks of one per workgroup) of a launch
void launch_barrier_reset(const Work& w, int lines, hipStream_t st);

// Band rules of the relaxation.
enum BandRule : int {
    BAND_PAPER = 0,      // Eq. upper_band / Eq. lower_band (relative change)
    BAND_FIXED_HALF = 1, // [max(1, floor((k+1)/2)), min(k, rho-1)] for 2 rho - 3 iterations
    BAND_JACOBI = 2,     // every topleset from 1; stop when no value changed
};

struct RunParams {
    int B, kmax_fixed, window;   // kmax_fixed 0: the rule's default per mesh
    int band_rule;
    long long N;
    float tol;
    const int* S;
    const float* upper;          // warm start: caller-order upper bound, or null
    bool certify;                // warm start: certify the bound (else trusted)
    float* out_d;
    double* out_d64;             // the double-precision run's output
    int* out_l;                  // labels (caller order), or null
    long long Stot;              // sources over the batch (labels)
    int jump_rounds;             // pointer-jumping rounds of the labels: ceil(log2(largest n)) + 1
    int ngroups;                 // groups of the launch (their classes head the queue array)
};

// cache: use the register-caching relaxation (single meshes); f64: the
// double-precision relaxation (no labels, no warm start, no cache); labels:
// Voronoi labels of the final map into p.out_l after the relaxation
hipError_t launch_run(const Work& w, const RunParams& p, bool labels, bool cache, bool f64, int g_run,
                      hipStream_t st);

// parents of the last labelled run in the caller's order (caller vertex
// ids; a source its own id, -1 where none)
hipError_t launch_parents_out(const Work& w, int B, long long N, int* out, hipStream_t st);

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
int max_coop_blocks_run(int cus, bool cache, bool rules);
int max_coop_blocks_run64(int cus, bool rules);

// farthest point sampling: argmax of the caller-order map of mesh 0, append
// to S, grow the mesh's source count; and the BFS + reorder alone (the
// incidence of the mesh is unchanged between samples)
hipError_t launch_fps_pick(const Work& w, const float* dist, int n, int* S, int slot, float* radius,
                           long long* step_stats, hipStream_t st);
hipError_t launch_prepare_bfs(const Work& w, const Sizes& z, const float* V, const int* S, int g_prep,
                              int n_one, int n_big, hipStream_t st);

// Lloyd step on Voronoi labels: cell moments over the faces, centroids, the
// nearest vertex of each cell
hipError_t launch_lloyd(const Work& w, const float* V, const int* F, int nv, int nf, const int* label,
                        const int* S_in, int m, int* S_out, double* centroid, hipStream_t st);

}  // namespace ptp
