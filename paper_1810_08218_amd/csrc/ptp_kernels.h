// Internal interface between the host API and the kernel sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ptp {

// Device workspace of one plan, carved from the caller's buffer.
struct Work {
    int* ctrl;          // C_WORDS control words
    int* level;         // [n]    hop distance, caller ids (-1 unreachable)
    int* perm;          // [n]    position -> caller id (the BFS queue)
    int* iperm;         // [n]    caller id -> position
    int* offsets;       // [n+2]  topleset starts in positions
    int* rowO;          // [n+1]  incidence CSR over caller ids
    int* faceO;         // [3f]   incident corners (3 * face + corner)
    int* cursor;        // [n]    fill cursors
    int* rowN;          // [n+1]  incidence CSR over positions
    int2* wedge;        // [3f]   opposite edge of each incident triangle, positions
    float4* xyz;        // [n]    coordinates by position (w unused)
    float* dist;        // [2n]   Jacobi double buffer
    int* lab;           // [2n]   label double buffer
    unsigned* bits;     // [2*nwords] frontier bitmaps
    int* cnt;           // [4*gmax] per-workgroup chunk counts
    int* retire;        // [n]    last iteration that updated each topleset
    int* scan_tmp;      // block sums of the scans
    unsigned* bar;      // [(gmax + 1) * 32] barrier lines (last one: release)
};

constexpr int kLayoutParts = 18;

struct Layout {
    size_t off[kLayoutParts];
    size_t total;
};

size_t work_layout(int n, int f, int gmax, Layout* L);
Work carve(void* base, int n, int f, int gmax, const Layout& L);

// prepare pipeline; every kernel after validation is gated on the status word
hipError_t launch_prepare(const Work& w, int n, int f, int m, const float* V, const int* F,
                          const int* S, int g_bfs, hipStream_t st);

// zero the barrier lines of a grid of g workgroups (before each persistent launch)
void launch_barrier_reset(const Work& w, int g, hipStream_t st);

struct RunParams {
    int n, m, rho, kmax, window;
    float tol;
    const int* S;
    float* out_d;
    int* out_l;
};

hipError_t launch_run(const Work& w, const RunParams& p, bool labels, int g_run, hipStream_t st);

// occupancy-bounded cooperative grid sizes
int max_coop_blocks_bfs(int cus);
int max_coop_blocks_run(int cus, bool labels);

}  // namespace ptp
