// Internal declarations shared by the host plan, the launchers and the
// kernels of the HIP SHT library.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "sht.h"

namespace sht {

// Legendre kernel geometry.  North rings form groups of 64 (one per lane of
// a wave); a wave owns R groups (R rings per lane).  Start indices of every
// l-chain are rounded down to a multiple of kChunk chain steps so that new
// lanes only join at chunk boundaries.
constexpr int kLanes = 64;
constexpr int kChunk = 8;
constexpr int kCoefPad = 2 * kChunk + 8;   // coefficient entries kept past l = L
constexpr int kDead = 0x3fffffff;          // start index of a chain that never
                                           // reaches the cutoff

// Bytes of the fixed device scratch behind sht_synthesis_noalloc.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// Run fn(i) for i in [0, n) on up to nthreads host threads (dynamic schedule).
void parallel_for(long n, int nthreads, void (*fn)(long, void *), void *ctx);

// Butterfly records (butterfly_plan.cpp builds them, butterfly.hip walks them).
constexpr int kBfMaxLv = 10;     // deepest level a plan may keep
constexpr int kBfTaskRings = 256; // rings of one residual wave task (up to four per lane)
constexpr int kBfPieceRings = 256; // rings of one forward residual piece (64, 128 or 256: one, two or four per lane)
constexpr int kBfNodeInts = 16;  // vin0, vin1, k0, k1, nd0, nd1, out, perm offset,
                                 // region flags, m, t, level, T offsets of both
                                 // children (64-bit, lo/hi)

// Long-double inputs of the butterfly precompute (from the plan build).
struct BflyInput {
    const long double *coefl;     // [entries][3] beta, alpha*beta, gamma
    const long double *start_ld;  // [(L+1)*2][2][n_north_pad] chain start values
    const long double *z2l;       // [n_north] z^2
};

struct BflyPlan {
    int built = 0;
    int K = 0;                        // columns: north rings
    long long ws_entries = 0;         // vector entries (2B values each) of the workspace
    int max_n = 0;                    // widest column set C of any pair node
    std::vector<int> depth;           // [(L+1)*2] levels kept per (m, t)
    long long n_tasks = 0;
    std::vector<int> res_task;        // [tasks][8] t, first row, end row, rings, output entry, m
    std::vector<int> res_lane;        // [tasks*256][2] ring, first row of the ring
    std::vector<double> res_val;      // [tasks*256][2] Legendre values at that row and the next
    std::vector<int> res_sub;         // [subtasks][8] the tasks cut into kBfPieceRings pieces for the
                                      // forward kernel: t, first row of the piece, end row,
                                      // rings, output entry, m, first lane record, 0
    int nbatch = 1;                   // orders m are run in batches m mod nbatch
    std::vector<int> batch_count;     // [nbatch] orders in each batch
    std::vector<long long> batch_task;  // [nbatch+1] residual task ranges
    std::vector<long long> batch_sub;   // [nbatch+1] sub-task ranges
    std::vector<long long> lv_off;    // [nbatch][kBfMaxLv+1] (+1) node ranges, deepest level first
    std::vector<int> lv_max_n;        // [nbatch][kBfMaxLv] widest column set of each range
    std::vector<int16_t> perm;        // per node and child: positions in C of the skeleton
                                      // columns (s order), then of the dense ones (d order)
    std::vector<int> node_i;          // [nodes][kBfNodeInts]
    std::vector<double> T;            // interpolation matrices, dense part, [s][d]
    long long T_entries = 0, res_elems = 0, n_nodes = 0, n_res_lanes = 0, n_units = 0;
    long long level_T[kBfMaxLv + 1] = {};      // dense entries of the pair nodes of each level
    long long level_units[kBfMaxLv + 1] = {};  // columns (output entries) of each level
    long long level_nodes[kBfMaxLv + 1] = {};  // pair nodes of each level
    // Level 1 of orders whose two parities both have levels runs fused with
    // the even/odd fold: units {even node, odd node, first ring, slot}; the
    // other level-1 nodes run alone and their orders are folded afterwards.
    std::vector<int> f1_unit, l1_plain, fold_slot;
    std::vector<long long> f1_off, l1_off, fold_off;  // [nbatch+1] ranges
    long long res_exec = 0;           // lane-steps the residual tasks execute
    long long depth_hist[kBfMaxLv + 1] = {};
    double build_seconds = 0.0;
    bool host_T_kept = true;
};

int interp_decomp(double *A, int r, int c, double tol, double abs_floor, std::vector<int> &piv,
                  std::vector<double> &T);

// Interpolation form of the Legendre phase (Sec. 3.3, Eq. 23): nodes at the
// roots of P~_N^m, N = m + t + 2 n_t, per (m, t) (interp_plan.cpp builds it,
// interp.hip applies it).
struct InterpPlan {
    int built = 0;
    std::vector<long long> node_off;  // [(L+1)*2 + 1] first node of (m, t)
    std::vector<double> x_hi, x_lo;   // [nodes] z_j^2 as a double-double
    std::vector<double> gam;          // [nodes] first-form weights gamma_j
    std::vector<double> lamN;         // [(L+1)*2][n_north_pad] P~_N^m(y_k), 0 where the chain is dead
    std::vector<int> sub;             // [pieces][8] node tasks in the residual kernel's format
    std::vector<int> lane;            // [pieces*kBfPieceRings][2] node, first row
    std::vector<double> val;          // [pieces*kBfPieceRings][2] chain values at that row and the next
    // nodes nearest the poles (sin(theta) below the plan's double-double
    // threshold) run a compensated chain instead: one wave of up to 64 nodes
    std::vector<int> dd_task;         // [tasks][8] t, m, chain length n, nodes, first entry, first lane, imin, 0
    std::vector<int> dd_lane;         // [tasks*64][2] node, first row
    std::vector<double> dd_val;       // [tasks*64][4] start values at that row and the next, hi and lo
    // rings closer to a node than the nodes' own precision allows for: both
    // parities are evaluated at the ring itself (extra node slots after the
    // n nodes of each (m, t), weight 0) and written over the interpolated
    // value: {m, ring, slot of t = 0, slot of t = 1} (-1: that chain is dead)
    std::vector<int> patch;           // [patches][4]
    long long nodes = 0, dd_nodes = 0, steps = 0, exec = 0, direct = 0;
    double build_seconds = 0.0;
};

struct RingClass {
    int lds_entries;              // complex entries of the FFT buffer (before padding)
    bool wrap = false;            // some ring has J/2 <= L (q staged through LDS)
    std::vector<int> rings;       // ring indices (host)
    int *d_rings = nullptr;       // device copy
};

}  // namespace sht

struct sht_plan_s {
    int L = 0, nside = 0, nrings = 0, n_north = 0, n_north_pad = 0, n_dd_pad = 0;
    double eps = 0.0;
    sht_plan_opts opts{};
    int device = -1;  // -1: host-only plan
    double build_seconds = 0.0;

    // ---- host tables --------------------------------------------------
    std::vector<double> z2_hi, z2_lo;          // [n_north_pad] z^2 of north rings
    std::vector<int> ring_J, ring_s;           // [nrings]
    std::vector<long long> ring_off;           // [nrings]
    std::vector<long long> coef_off;           // [L+1] entry offset of order m
    std::vector<double> coef_hi, coef_lo;      // 4 doubles per entry
    std::vector<int> start_idx;                // [(L+1)*2][n_north_pad]
    std::vector<double> start_val;             // [(L+1)*2][2][n_north_pad]
    std::vector<double> start_lo;              // [(L+1)*2][2][n_dd_pad]
    std::vector<int> grp_lo, grp_hi;           // [(L+1)][n_north_pad/64]
    int n_dd_rings = 0, n_dd_groups = 0;
    int rings_per_lane = 2;                    // R of the FP64 Legendre waves
    int ring_threads = 1024;                   // workgroup size of the ring kernel
    long long n_step = 0, n_step_exec = 0, n_step_dd = 0, n_step_lanes = 0;

    // ring FFT tables
    int tw_log = 0;                            // twiddle table covers 2^tw_log
    std::vector<double> tw;                    // [2^(tw_log-1)][2]
    std::vector<int> ring_M;                   // [nrings] 0 = radix-2 size J/2, else Bluestein size
    std::vector<long long> ring_bs_off;        // [nrings] offset (complex entries) of the chirp spectrum
    std::vector<double> bs_table;              // chirp spectra, bit-reversed, scaled by 1/M
    std::vector<double> chirp;                 // exp(+i pi k^2 / n), k < n, per distinct Bluestein n
    std::vector<long long> ring_chirp_off;     // [nrings] offset (complex entries) into chirp
    std::vector<sht::RingClass> classes;

    // polarized synthesis near the poles: north rings [0, pol_n) (and their
    // mirrors) whose sin(theta) is below the threshold where the reduction
    // to scalar transforms loses accuracy; per ring z, sin(theta/2),
    // cos(theta/2) as double-double pairs; per (m, s = +2, -2) the value of
    // _s lambda at l0 = max(m, 2) without its powers of sin and cos(theta/2),
    // as a double-double mantissa times 2^exp (sign included)
    int pol_n = 0;
    std::vector<double> pol_ring;              // [pol_n][6]
    std::vector<double> pol_K;                 // [(L+1)*2][4] hi, lo, exp, 0

    // ---- device copies ------------------------------------------------
    double *d_z2_hi = nullptr, *d_z2_lo = nullptr;
    int *d_ring_J = nullptr, *d_ring_s = nullptr, *d_ring_M = nullptr;
    long long *d_ring_off = nullptr, *d_ring_bs_off = nullptr, *d_coef_off = nullptr;
    double *d_coef_hi = nullptr, *d_coef_lo = nullptr;
    int *d_start_idx = nullptr;
    double *d_start_val = nullptr, *d_start_lo = nullptr;
    int *d_grp_lo = nullptr, *d_grp_hi = nullptr;
    double *d_tw = nullptr, *d_bs_table = nullptr, *d_chirp = nullptr;
    long long *d_ring_chirp_off = nullptr;
    double *d_pol_ring = nullptr, *d_pol_K = nullptr;
    size_t device_bytes = 0;

    // ---- butterfly (eps > 0) ------------------------------------------
    sht::BflyPlan bf;
    int *d_bf_res_task = nullptr, *d_bf_res_lane = nullptr, *d_bf_res_sub = nullptr;
    double *d_bf_res_val = nullptr, *d_bf_T = nullptr;
    float *d_bf_T32 = nullptr;
    double *d_bf_Tt = nullptr;  // transposed copies for the adjoint (store_transpose)
    float *d_bf_Tt32 = nullptr;
    int16_t *d_bf_perm = nullptr;
    int *d_bf_node_i = nullptr;
    int *d_bf_f1_unit = nullptr, *d_bf_l1_plain = nullptr, *d_bf_fold_slot = nullptr;

    // ---- interpolation to Legendre-root nodes (opts.interp) -------------
    sht::InterpPlan ip;
    long long *d_ip_node_off = nullptr;
    double *d_ip_x_hi = nullptr, *d_ip_x_lo = nullptr, *d_ip_gam = nullptr, *d_ip_lamN = nullptr;
    int *d_ip_sub = nullptr, *d_ip_lane = nullptr, *d_ip_dd_task = nullptr, *d_ip_dd_lane = nullptr;
    double *d_ip_val = nullptr, *d_ip_dd_val = nullptr;
    int *d_ip_patch = nullptr;

};

namespace sht {

// Device address of the fixed scratch on device `dev` (current), looked up
// once per device (noalloc.hip).
int noalloc_scratch(int dev, void **out);

// Argument block of the brute-force Legendre waves (legendre.hip): one
// plan, one pass of up to 4 maps.
struct LegArgs {
    const double *__restrict__ z2_hi;
    const double *__restrict__ z2_lo;
    const long long *__restrict__ coef_off;
    const double *__restrict__ coef_hi;
    const double *__restrict__ coef_lo;
    const int *__restrict__ start_idx;
    const double *__restrict__ start_val;
    const double *__restrict__ start_lo;
    const int *__restrict__ grp_lo;
    const int *__restrict__ grp_hi;
    const double *__restrict__ alm;
    double *__restrict__ q;
    int L, nrings, n_north, np, n_dd_pad, ng;
    int nmaps, map0;  // map stride of alm/q and first map of this pass
    int dd_groups;    // 64-ring groups run in double-double (from the pole)
    int fp_blocks;    // FP64 ring blocks of R groups after them
};

// Argument block of the ring FFT workgroups (ring.hip): one plan, one ring
// size class.
struct RingArgs {
    const int *__restrict__ rings;
    int count;
    const int *__restrict__ ring_J;
    const int *__restrict__ ring_s;
    const int *__restrict__ ring_M;
    const long long *__restrict__ ring_off;
    const long long *__restrict__ ring_bs_off;
    const double2 *__restrict__ tw;
    int tw_log;
    const double2 *__restrict__ bs_table;
    const double2 *__restrict__ chirp;
    const long long *__restrict__ ring_chirp_off;
    const double2 *__restrict__ q;
    double *__restrict__ map;
    int L, nrings, nmaps;
    long long npix;
    int fft_entries;  // padded FFT buffer entries of this launch's class
    int stage;        // LDS entries past the FFT buffer (wrapped rings' reduction room)
    int mpw;          // maps of one ring per workgroup (1, 2 or 4; divides nmaps)
    // adjoint direction: pixel values in, weighted phases ybar out
    const double *__restrict__ map_in;
    double2 *__restrict__ ybar;
    double wpos;      // weight of m >= 1 (2: transpose of synthesis, 1: Y^dagger)
};

// Host plan construction (plan.cpp, butterfly_plan.cpp).
int build_host_tables(sht_plan_s *p);
int build_butterfly(sht_plan_s *p, const BflyInput &in);
int build_interp(sht_plan_s *p, const BflyInput &in);
int build_pol_tables(sht_plan_s *p);
int pol_column_host(const sht_plan_s *p, int m, int s, int k, double *out);
// polarized synthesis (pol.hip)
size_t pol_alm_bytes(const sht_plan_s *p, int nmaps);
hipError_t launch_pol_prep(const sht_plan_s *p, int nmaps, const double *E, const double *B, double *alm6,
                           hipStream_t st);
hipError_t launch_pol_combine(const sht_plan_s *p, int nmaps, const double *q6, double *q2, hipStream_t st);
hipError_t launch_pol_polar(const sht_plan_s *p, int nmaps, const double *E, const double *B, double *q2,
                            hipStream_t st);
int interp_apply_host(const sht_plan_s *p, int m, int t, const double *x, double *y);
int butterfly_apply_host(const sht_plan_s *p, int m, int t, const double *x, double *y);
int upload_tables(sht_plan_s *p);
void free_device_tables(sht_plan_s *p);

// Launchers (kernels_*.hip).  All enqueue on `stream` and return a HIP error.
hipError_t launch_legendre(const sht_plan_s *p, int nmaps, const double *alm, double *q,
                           hipStream_t stream);
hipError_t launch_ring_synthesis(const sht_plan_s *p, int nmaps, const double *q, double *map,
                                 hipStream_t stream);
hipError_t launch_ring_analysis(const sht_plan_s *p, int nmaps, const double *map, double *ybar,
                                double wpos, hipStream_t stream);
hipError_t launch_legendre_adjoint(const sht_plan_s *p, int nmaps, const double *ybar, double *g,
                                   hipStream_t stream);
// Butterfly Legendre phase (eps > 0 plans): alm -> folded q, like
// launch_legendre; scratch holds ws_entries vector entries of up to 16
// doubles (FP64) or floats (FP32).
size_t bf_scratch_bytes(const sht_plan_s *p, int nmaps, int fp32);
// stage_events: NULL or the caller's 2*SHT_NSTAGES event handles; the
// residual and level launches are bracketed for one-batch plans.
hipError_t launch_butterfly(const sht_plan_s *p, int nmaps, const double *alm, double *q, void *scratch,
                            int fp32, hipStream_t stream, void *const *stage_events = nullptr);
// Work-queue batches on the butterfly path (butterfly.hip): the argument
// block of one pass (bf_args_bytes() bytes, written to out), one stage
// launch over items {pass, index} (stage 0 residual pieces, 1 level nodes,
// 2 fused level-1 units, 3 fold blocks), and a node's LDS bytes.
size_t bf_args_bytes(int fp32);
void bf_queue_args(const sht_plan_s *p, int nmaps, int map0, int nb, int fp32, const double *alm, double *q, void *ws,
                   void *out);
hipError_t launch_bf_queue_stage(int stage, int nb, int fp32, const void *args, const int2 *items, long long n,
                                 size_t lds, hipStream_t st);
size_t bf_level_lds_bytes(int n, int nb, int fp32);
// Interpolation form (opts.interp plans): alm -> folded q through the
// Legendre-root nodes; scratch holds ip.nodes entries of up to 8 doubles.
size_t interp_scratch_bytes(const sht_plan_s *p, int nmaps);
hipError_t launch_interp(const sht_plan_s *p, int nmaps, const double *alm, double *q, void *scratch,
                         hipStream_t stream);
// Its transpose: unfolded ybar (ring-major, like q) -> g (written whole),
// with the same scratch.
hipError_t launch_butterfly_adjoint(const sht_plan_s *p, int nmaps, const double *ybar, double *g, void *scratch,
                                    int fp32, hipStream_t stream);
// Work-queue batch pieces (legendre.hip, ring.hip): the argument block of
// one pass, the persistent Legendre launch over a sorted item list (items
// {pass, m, ring block, maps}; counter is device memory the launch resets),
// and one ring-queue launch per ring size class (items {argument block,
// item of that class}).  The Legendre items come in one list per XCD.
LegArgs leg_args(const sht_plan_s *p, int nmaps, int map0, int R, const double *alm, double *q);
// Work-queue batches on the brute-force path: one persistent launch per wave
// shape (0, 1: compensated waves of 2 or 1 maps; 2, 3, 4: FP64 waves of 4,
// 2 or 1 maps).
constexpr int kQueueShapes = 5;
// Internal streams for fork/join inside one call (batch.cpp).
constexpr int kMaxStreams = 8;
int pool_streams(int dev, hipStream_t *out);
int queue_shape(bool dd, int nb);
hipError_t legendre_queue_grid(int shape, int rings_per_lane, int *grid);
// items {pass, m, ring block, first map}: per shape eight lists back to back,
// cut into chunks; chunk c covers items [chunk_off[c], chunk_off[c+1]) and
// list x of shape v the chunks [list_off[9v+x], list_off[9v+x+1]); counter:
// 5 x 8 x 16 unsigned of device memory, cleared by launch_queue_reset before
// the shapes' launches; grid: waves of the shape's launch (0: no items).
hipError_t launch_queue_reset(unsigned *counter, hipStream_t st);
hipError_t launch_legendre_queue(int shape, const LegArgs *passes, const int4 *items, const unsigned *chunk_off,
                                 const unsigned *list_off, unsigned *counter, int rings_per_lane, int grid,
                                 hipStream_t st);
RingArgs ring_args(const sht_plan_s *p, int nmaps, const double *q, double *map);
size_t ring_class_shape(int lds_entries, bool wrap, int T, int *fft_entries, int *stage);
int ring_maps_per_wg(int lds_entries, int nmaps);
hipError_t launch_ring_queue(int T, const RingArgs *args, const int2 *items, long long nitems, size_t lds,
                             hipStream_t st);
hipError_t ring_queue_prepare(int T);
// y = alpha x + beta y over n doubles (beta = 0: y = alpha x).
hipError_t launch_axpby(double *y, const double *x, double alpha, double beta, long long n, hipStream_t st);
// Device-side transposed copies of the interpolation matrices (d_bf_Tt and,
// when the FP32 copy exists, d_bf_Tt32) from the uploaded ones; nT entries,
// nnodes pair nodes.  Adds the allocated bytes to *bytes.
hipError_t bf_store_transposed(sht_plan_s *p, size_t nT, size_t nnodes, size_t *bytes);

}  // namespace sht
