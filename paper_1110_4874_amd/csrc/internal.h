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

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// Run fn(i) for i in [0, n) on up to nthreads host threads (dynamic schedule).
void parallel_for(long n, int nthreads, void (*fn)(long, void *), void *ctx);

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
    std::vector<sht::RingClass> classes;

    // ---- device copies ------------------------------------------------
    double *d_z2_hi = nullptr, *d_z2_lo = nullptr;
    int *d_ring_J = nullptr, *d_ring_s = nullptr, *d_ring_M = nullptr;
    long long *d_ring_off = nullptr, *d_ring_bs_off = nullptr, *d_coef_off = nullptr;
    double *d_coef_hi = nullptr, *d_coef_lo = nullptr;
    int *d_start_idx = nullptr;
    double *d_start_val = nullptr, *d_start_lo = nullptr;
    int *d_grp_lo = nullptr, *d_grp_hi = nullptr;
    double *d_tw = nullptr, *d_bs_table = nullptr;
    size_t device_bytes = 0;

};

namespace sht {

// Host plan construction (plan.cpp).
int build_host_tables(sht_plan_s *p);
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

}  // namespace sht
