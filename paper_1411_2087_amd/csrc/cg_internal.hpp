// Solver state and helpers shared by the CG sources.
#pragma once

#include "dslash_core.hpp"

namespace hisq {

enum { CG_RUNNING = 0, CG_CONVERGED = 1, CG_BREAKDOWN = 2, CG_STALLED = 3 };

// Gate of the kernels of a solver iteration: closed when the solve is done
// or a reliable update is pending.  The iteration pauses there; the host
// runs the update outside the captured graph at its next state check and
// the iterations resume.
enum { GATE_PAUSE = 3 };
__device__ __forceinline__ bool paused(const SolverFlags &f) { return f.done || f.reliable; }
__device__ __forceinline__ bool solver_gate_closed(const SolverFlags *f, int gate)
{
    return gate == GATE_PAUSE ? paused(*f) : gate_closed(f, gate);
}
// Device-resident scalars of one solve.  `flags` comes first: kernels gate on it.
struct CGState {
    SolverFlags flags;
    int iter;        // iterations completed
    int nupdates;    // reliable updates done
    double tol2;     // tol^2
    double bb;       // |b|^2
    double stop2;    // tol^2 |b|^2
    double m4;       // 4 m^2
    double delta2;   // reliable-update threshold delta^2
    double rr;       // |r|^2 of the current iterate (inner residual in mixed modes)
    double rr_new;   // |r|^2 after the last update
    double rr_true;  // last FP64 true residual |b - A x|^2
    double maxrr;    // max |r_inner|^2 since the last reliable update
    double alpha, beta, pAp;
    // stagnation watch of the mixed solver (reliable updates that do not
    // reduce the true residual, or an inner solve that stops triggering them)
    double rr_upd;   // true |r|^2 at the last reliable update (or the start)
    int last_upd;    // iteration of the last reliable update
    int first_gap;   // iterations from the start to the first reliable update
    int poor;        // consecutive reliable updates that did not halve |r|
    int pad_;
};

// Algorithmic bytes per site of the byte model of every solver's bytes_moved:
// the 16 link matrices of one Dslash in precision `prec` (a two-row long
// matrix is 96, 48 or 28 bytes) and one colour vector of its vector type.
inline double link_bytes_site(int prec)
{
    switch (prec) {
    case HISQ_F64: return 16 * 144.0;
    case HISQ_F32: return 16 * 72.0;
    case HISQ_F16S:
    case HISQ_I16S: return 16 * 40.0;
    case HISQ_F64C: return 8 * 144.0 + 8 * 96.0;
    case HISQ_F32C: return 8 * 72.0 + 8 * 48.0;
    default: return 8 * 40.0 + 8 * 28.0;  // HISQ_I16SC
    }
}
inline double vec_bytes(int prec) { return (prec == HISQ_F64 || prec == HISQ_F64C) ? 48.0 : 24.0; }

// Scratch of the standalone dot product: the per-workgroup partials of the
// first stage (at most BLAS_MAX_BLOCKS workgroups, striding over the vectors)
// and the result.  dot_on launches the two stages on `s` and copies the
// result to out_host (synchronises `s`).
constexpr int BLAS_MAX_BLOCKS = 1024;
constexpr size_t DOT_PART_BYTES = 2 * sizeof(double) * BLAS_MAX_BLOCKS;
constexpr size_t DOT_WS_BYTES = DOT_PART_BYTES + 256;
int dot_on(const void *x, const void *y, long long n, int prec, double out_host[2], char *ws, hipStream_t s);

int blas_blocks(long long n);
size_t cg_partials_count(const Geom &g);
size_t cg_multi_workspace_bytes(const Geom &g, int nrhs, int mode);
size_t fcg_ws_bytes(const Geom &g, int channels);
size_t fat_paths_ws_bytes(const int dims[4]);  // links.hip
// Pinned host mirrors of the solvers' device states: one block per thread,
// allocated by the first solve on the thread and kept, so no solve allocates
// or frees pinned memory (hipHostFree would synchronise the device).  Slots:
// fcg_solve keeps its state live while its plain-CG fallback uses PIN_CG.
enum { PIN_CG = 0, PIN_MULTI = 1, PIN_FCG = 2, PIN_SLOTS = 3 };
constexpr size_t PIN_SLOT_BYTES = 16384;
void *pinned_slot(int slot);
inline CGState *pinned_state() { return (CGState *)pinned_slot(PIN_CG); }
hipStream_t capture_stream();
hisq_cg_opts resolve_opts(const hisq_cg_opts *opts, const Geom &g);

}  // namespace hisq
