// Internal declarations of libddm (HIP, gfx950).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ddm.h"

namespace ddm {

// Device-side descriptor of one subdomain (extended box E_a of Sec. 3.1).
struct SubDesc {
    int lo[3], hi[3];      // extended box, physical node indices (unused axes: 0)
    int clo[3], chi[3];    // core box
    int n[3];              // box extents (1 on unused axes)
    int sid[3];            // subdomain multi-index
    long long off;         // packed offset (elements per RHS)
    long long nloc;        // box size
    int nb;                // number of blocks (grid lines / planes) along the last axis
    int mid;               // twist block: blocks < mid are eliminated from the first block
                           // on, blocks > mid from the last block on; mid = nb - 1 gives
                           // the one-directional factorisation
    int bs;                // block size (n[0] in 2D, n[0]*n[1] in 3D)
    int ld;                // column stride of the stored block inverses: bs, or bs + 1 for
                           // odd complex64 blocks (16-byte aligned pairs of rows)
    int mpad;              // matrix-core layout of the inverses: columns rounded up to a
                           // whole operand group (8 for complex64, 4 for complex128);
                           // 0 where that layout does not apply (bs > 256)
    long long foff;        // factor offset (elements)
    int coff[3];           // offsets of this box's per-axis coefficient tables
    int nbr[26];           // neighbour ids for the 26 offsets (-1: none)
    int lag[26];           // lag = number of differing axes
};

// Per-node 1D coefficients of the PML operator along one axis:
// (T u)(x) = cp (u(x+1) - u(x)) - cm (u(x) - u(x-1)),
// cp = 1/(alpha(x) alpha(x+1/2) h^2), cm = 1/(alpha(x) alpha(x-1/2) h^2).
struct Coef {
    double2 cp, cm;
};

// One GEMV work item of the substitution kernels: rows [r0, r0 + 64) of the
// blocks of subdomain a.
struct SolveItem {
    int a, r0;
};

// Per axis and global index: the (at most two) subdomain coordinates along
// the axis whose box holds the index with a non-zero cut-off factor b(m), in
// increasing order, with the local coordinate and the box extent.
struct AxisOwn {
    double beta[2];
    int i[2];
    int lc[2];
    int n[2];
    int cnt;
    int pad;
};

struct Plan {
    int dim = 2;
    int M[3] = {0, 0, 0}, N[3] = {1, 1, 1}, C[3] = {1, 1, 1};
    int G[3] = {1, 1, 1}, glo[3] = {0, 0, 0};
    int n_pml = 0, n_ov = 0;
    double h = 0, sigma0 = 0;
    long long nglob = 0, etot = 0;
    int nsub = 0;
    int ring = 3;               // generations of local solutions kept (lags)
    int bs_max = 0, nb_max = 0;
    long long fel = 0;          // factor elements
    std::vector<SubDesc> subs;
    std::vector<Coef> coef;     // local tables (per subdomain, per axis)
    std::vector<Coef> gcoef;    // global tables per axis (offsets gcoff)
    int gcoff[3] = {0, 0, 0};
    std::vector<int2> strip;    // (subdomain, local node) of every node in a transfer strip
    std::vector<AxisOwn> aown;  // per axis, per global index: boxes with a non-zero cut-off
    int aoff[3] = {0, 0, 0};
    std::vector<double> btab;   // side cut-off factor b(m), m = 0 .. n_ov
    std::vector<SolveItem> items;
    bool twisted = false;           // factor layout: both-ends elimination
    bool mma = false;               // inverses stored in matrix-core operand order (else column-major)
    int mpad_max = 0;               // largest SubDesc.mpad
    int ncu = 256;                  // compute units of the device: co-residency bound of the chain launches
    std::vector<double> w_el_by_l;  // sum over subdomains with > l blocks of bs^2
    std::vector<double> v_el_by_l;  // same, of bs
};

int build_plan(const ddm_problem *p, Plan *plan, std::string *err);
// Device address of the library's static scratch array on device dev (which
// must be current); resolved once per device.  Returns hipSuccess or the
// error of the symbol lookup.
hipError_t scratch_init(int dev);
// choose the elimination layout (sets mid of every subdomain)
void plan_set_twist(Plan *plan, bool twisted);
bool plan_twist_fits(const Plan &P);

}  // namespace ddm

struct ddm_handle {
    ddm_problem prob;
    ddm::Plan plan;
    hipStream_t stream = nullptr;
    int device = 0;                 // HIP device current at ddm_setup
    std::string err;
    int nrhs_max = 0;
    bool mixed = false;
    bool factored = false;
    // device tables
    ddm::SubDesc *d_subs = nullptr;
    ddm::Coef *d_coef = nullptr, *d_gcoef = nullptr;
    ddm::AxisOwn *d_aown = nullptr;
    int2 *d_strip = nullptr;
    double *d_btab = nullptr;
    double *d_k2 = nullptr;
    ddm::SolveItem *d_items = nullptr;
    // factors: complex128 (FP64) or complex64 (MIXED), column-major blocks
    void *d_W = nullptr;
    void *d_scratch = nullptr;      // factorisation workspace (freed after ddm_factor)
    int *d_flags = nullptr;         // per-subdomain status flags
    // step workspaces, element type T (double2 or float2), nrhs_max * etot each
    void *d_g = nullptr;
    int g_clean_rows = 0;           // RHS rows of d_g known to be zero outside the transfer strips
    void *d_ring[4] = {nullptr, nullptr, nullptr, nullptr};
    // FP64 global workspaces
    double2 *d_r = nullptr;         // residual / operator output, nrhs_max * nglob
    double2 *d_wide = nullptr;      // packed complex128 scratch for the ABI row entries
    double *d_part = nullptr;       // norm partial sums
    size_t part_cap = 0;            // doubles in d_part
    double *d_norm = nullptr;       // per-RHS norms (device)
    double *h_norm = nullptr;       // pinned host copy
    int *d_active = nullptr;        // per-RHS flags for the assembly
    int nblk_norm = 0;
    size_t bytes = 0;               // device bytes held (every allocation counted)
    size_t peak_bytes = 0;          // most device bytes held at once
    // FGMRES storage (allocated on first use)
    double2 *d_V = nullptr, *d_Z = nullptr;
    int krylov_m = 0, krylov_nrhs = 0;
    double2 *d_dots = nullptr;      // (m+1) * nrhs dot products
    double2 *h_dots = nullptr;      // pinned
    double2 *d_coef_y = nullptr;    // Krylov combination coefficients
    // substitution kernel variant (autotuned) and persistent-launch sync state
    int solve_variant = 0;
    int chain_tile = 0;             // chain variant, batches of > 4 RHS: RHS tile 4, 8 or 16 (0 = by batch size)
    int *d_sync = nullptr;          // per parallel RHS tile of the matrix-core substitution: 2 nsub
                                    // meeting flags and 2 nsub read-done flags (the chain kernels use
                                    // the first tile's); then 1 abort flag
    int sync_tiles = 1;             // RHS tiles d_sync has flags for: ceil(nrhs_max / 16)
    int *d_sync2 = nullptr;         // split substitution: 4 nsub meeting, 4 nsub exchange and
                                    // 4 nsub read-done flags
    void *d_xbuf = nullptr;         // split substitution: double-buffered partial-sum exchange
    int spin_limit = 1 << 22;
    int transfer_form = 0;          // DDM_TRANSFER_DIRECT / DDM_TRANSFER_PHI
    // continuous batching: per-slot step counts (-1 = free), the handle's
    // global step counter drives the ring phase
    std::vector<int> slot_steps;
    long long slot_global = 0;
    bool slots_dirty = false;       // d_active needs an upload
    // hipGraph capture of the stationary DDM step (one graph per ring phase)
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t step_graph[4] = {nullptr, nullptr, nullptr, nullptr};
    int step_graph_nrhs[4] = {0, 0, 0, 0};
    double2 *d_fin = nullptr, *d_uin = nullptr;  // handle-owned f and u of the graph path
    long graph_launches = 0;
    // per-launch HIP event profiling (ddm_profile_enable)
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    struct ProfRec { hipEvent_t a, b; int cls; double bytes; };
    std::vector<ProfRec> prof_recs;
};

namespace ddm {

// sticky abort flag of the bounded waits in the substitution kernels
inline int *abort_flag_ptr(ddm_handle *h) { return h->d_sync + (size_t)4 * h->plan.nsub * h->sync_tiles; }

// RHS tiles of 16 whose flags d_sync holds for a handle of nrhs_max RHS
inline int sync_tiles_for(int nrhs_max) { return nrhs_max > 16 ? (nrhs_max + 15) / 16 : 1; }

// Bracket one launch with a pair of events when profiling is on.
struct ProfScope {
    ddm_handle *h;
    int cls;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    // on = false: never profile (the allocation-free entry points create no events)
    ProfScope(ddm_handle *h_, int cls_, double bytes_, bool on = true);
    ~ProfScope();
};

// ---- launchers (all enqueue on h->stream; return hipError_t) ----
hipError_t launch_apply(ddm_handle *h, const double2 *u, double2 *out, int nrhs);
hipError_t launch_residual(ddm_handle *h, const double2 *f, const double2 *u, double2 *r, int nrhs,
                           double *d_rn2, double *d_fn2);
// the same with the block partial sums (2 nrhs stencil_blocks doubles, every
// entry written before it is read) in a buffer of the caller's
hipError_t launch_residual_parts(ddm_handle *h, const double2 *f, const double2 *u, double2 *r, int nrhs,
                                 double *part, double *d_rn2, double *d_fn2, bool profile = true);
hipError_t launch_norm2(ddm_handle *h, const double2 *x, long long n, int nrhs, long long ld, double *d_out);

template <typename TIN, typename TOUT>
hipError_t launch_restrict(ddm_handle *h, const TIN *f, TOUT *g, int nrhs);
template <typename TIN, typename TOUT>
hipError_t launch_transfer(ddm_handle *h, const TIN *l1, const TIN *l2, const TIN *l3, TOUT *g, int nrhs,
                           const double2 *rcorr = nullptr);
template <typename TIN>
hipError_t launch_assemble(ddm_handle *h, const TIN *U, double2 *u, int nrhs, bool accumulate,
                           const int *d_active);

template <typename T>
hipError_t launch_factor(ddm_handle *h, void *ws);
// device workspace of the factorisation (allocated for ddm_factor only)
size_t factor_ws_bytes(const Plan &P);
template <typename T>
hipError_t launch_local_solve(ddm_handle *h, const T *g, T *x, int nrhs);

// substitution variants
enum { kSolvePerLine = 0, kSolveChain = 1, kSolveChain2 = 2, kSolveMma = 3, kSolveNVariants = 4 };
// the matrix-core substitution reads the inverses in its own operand order:
// a handle's stored layout follows its variant (P.mma == (variant == kSolveMma))
constexpr int kMmaMaxBs = 256;
bool solve_variant_ok(const Plan &P, int variant);
// matrix-core substitution (ddm_solve_mma.hip): applies to blocks of at most
// kMmaMaxBs unknowns (and, two-ended, one resident workgroup per chain);
// needs the inverses in its operand order (P.mma)
bool mma_fits(const Plan &P);
template <typename T2>
hipError_t run_mma(ddm_handle *h, const T2 *g, T2 *x, int nrhs);
// right-hand sides per handle from which the matrix-core substitution is the default
constexpr int kMmaMinRhs = 8;

// XCDs of the chip: workgroups are placed on them round-robin by index
constexpr int kXcds = 8;
// blocks of the row-per-block stencil launches: grid rows padded to a
// multiple of the XCD count
inline int stencil_blocks(const Plan &P) { return (P.G[1] * P.G[2] + kXcds - 1) / kXcds * kXcds; }
// The assembly kernel gives every global node a thread: a grid row is cut
// into pieces of kRowPiece nodes, one workgroup each.
constexpr int kRowPiece = 256;
inline int row_pieces(const Plan &P) { return (P.G[0] + kRowPiece - 1) / kRowPiece; }
size_t chain2_xbuf_bytes(const Plan &P);
bool chain2_fits(const Plan &P);

hipError_t launch_convert_c128_to_c64(const double2 *in, float2 *out, long long n, hipStream_t s);
hipError_t launch_convert_c64_to_c128(const float2 *in, double2 *out, long long n, hipStream_t s);
hipError_t launch_fill_zero(void *p, long long bytes, hipStream_t s);

// Krylov helpers (FP64 complex, batched over RHS; vectors of length n, RHS stride ld)
hipError_t launch_dots(const double2 *V, int nvec, long long vstride, const double2 *w, long long n, int nrhs,
                       long long ld, double2 *d_out, double *d_part, int nblk, hipStream_t s);
hipError_t launch_axpy_multi(double2 *w, const double2 *V, int nvec, long long vstride, const double2 *coef,
                             double sign, long long n, int nrhs, long long ld, hipStream_t s);
hipError_t launch_scale(double2 *y, const double2 *x, const double *scale, long long n, int nrhs, long long ld,
                        hipStream_t s);

}  // namespace ddm
