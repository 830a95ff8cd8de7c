// Brute-force Legendre phase (Wavemoth paper, Sec. 2.4 Eqs. 12-14 and
// App. A.2 Eqs. A1-A2), for gfx950.
//
//   q_m(+-z_k) = q^even_m(z_k) +- q^odd_m(z_k),
//   q^t_m(z)   = sum_i P~_{m+t+2i}^m(z) a_{m+t+2i, m}
//
// One wavefront handles one order m and a block of 64 x R north rings;
// every lane owns R rings (R = 1, 2 or 4, a plan parameter) and runs both
// parity chains of the two-step recurrence for them.  The recurrence coefficients
// and the a_lm of the current l are the same for every lane, so they are
// read as wave-uniform (scalar) loads and used straight from SGPRs; P~ never
// leaves VGPRs (the GPU form of the paper's register-resident SSE kernel).
// The even/odd fold of Eqs. 13-14 is fused into the store: each lane writes
// ring k and its mirror 4N-2-k.
//
// Chains start at the plan's precomputed values (first l above the cutoff,
// rounded down to a multiple of kChunk chain steps), so a lane joins the
// wave-uniform l loop only at chunk boundaries.  Ring blocks nearest the
// poles, where a z-based FP64 recurrence loses ~l eps / sin(theta), run the
// same recurrence in double-double arithmetic.
#include "ddmath.h"
#include "internal.h"

namespace sht {



// One wave: order m, rings of the 64-ring groups g0 .. g0+R-1 (R per lane).
// Groups at or past a.ng do not exist (partial last block) and are skipped.
template <int NB, int R, bool DD>
__device__ __forceinline__ void legendre_wave(const LegArgs &a, const int m, const int g0) {
    const int lane = threadIdx.x;
    const int L = a.L;

    int k[R];
    bool gv[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        gv[r] = g0 + r < a.ng;
        k[r] = (g0 + r) * kLanes + lane;
    }

    // wave-uniform chain range of this block
    int lo = kDead, hi = -1;
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (!gv[r]) continue;
        lo = min(lo, a.grp_lo[(size_t)m * a.ng + g0 + r]);
        hi = max(hi, a.grp_hi[(size_t)m * a.ng + g0 + r]);
    }
    const int n0 = (L - m) / 2 + 1;                    // even chain length
    const int n1 = (L - m >= 1) ? (L - m - 1) / 2 + 1 : 0;  // odd chain length

    double accE_r[R][NB], accE_i[R][NB], accO_r[R][NB], accO_i[R][NB];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int b = 0; b < NB; b++) accE_r[r][b] = accE_i[r][b] = accO_r[r][b] = accO_i[r][b] = 0.0;

    if (lo < n0) {
        double z2h[R], z2l[R];
        int sid[R][2];
        dd p0[R][2], p1[R][2];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int kk = gv[r] ? k[r] : 0;
            z2h[r] = a.z2_hi[kk];
            z2l[r] = DD ? a.z2_lo[kk] : 0.0;
#pragma unroll
            for (int t = 0; t < 2; t++) {
                size_t row = (size_t)(2 * m + t);
                sid[r][t] = gv[r] ? a.start_idx[row * a.np + kk] : kDead;
                p0[r][t] = {0.0, 0.0};
                p1[r][t] = {0.0, 0.0};
            }
        }
        const long long cbase = a.coef_off[m];
        const double *__restrict__ ch = a.coef_hi + 4 * cbase;
        const double *__restrict__ cl = a.coef_lo + 4 * cbase;
        const size_t aoff = (size_t)m * (2 * L + 3 - m) / 2;
        const double *__restrict__ al = a.alm + 2 * (aoff * a.nmaps + a.map0);
        const int astride = 2 * a.nmaps;  // doubles between consecutive l

        auto inject = [&](int c) {
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int t = 0; t < 2; t++)
                    if (sid[r][t] == c) {
                        // start values are read when the chain joins (once per
                        // chain), not kept in registers for the whole wave
                        const size_t row = (size_t)(2 * m + t);
                        const int kk = k[r];
                        p0[r][t].h = a.start_val[(row * 2 + 0) * a.np + kk];
                        p1[r][t].h = a.start_val[(row * 2 + 1) * a.np + kk];
                        p0[r][t].l = DD ? a.start_lo[(row * 2 + 0) * a.n_dd_pad + kk] : 0.0;
                        p1[r][t].l = DD ? a.start_lo[(row * 2 + 1) * a.n_dd_pad + kk] : 0.0;
                    }
        };

        // operands of chain step i (the same for every lane: scalar loads)
        struct Ops {
            double be, abe, ge, bo, abo, go;
            double er[NB], ei[NB], orr[NB], oi[NB];
        };
        auto load_ops = [&](int i, bool odd_ok) {
            Ops o;
            // entries l = m + 2i + 2 (even chain) and the next one (odd chain)
            const double4 *ce = reinterpret_cast<const double4 *>(ch) + (2 * i + 2);
            const double4 e4 = ce[0], o4 = ce[1];
            o.be = e4.x;
            o.abe = e4.y;
            o.ge = e4.z;
            o.bo = o4.x;
            o.abo = o4.y;
            o.go = o4.z;
            const double *ape = al + (size_t)(2 * i) * astride;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                o.er[b] = ape[2 * b];
                o.ei[b] = ape[2 * b + 1];
                o.orr[b] = odd_ok ? ape[astride + 2 * b] : 0.0;
                o.oi[b] = odd_ok ? ape[astride + 2 * b + 1] : 0.0;
            }
            return o;
        };

        // one chain step i for both parities: accumulate P(i) a_l, advance
        auto compute = [&](const Ops &o, int i) {
            if constexpr (!DD) {
                (void)i;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const double pe = p0[r][0].h, po = p0[r][1].h;
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        accE_r[r][b] = __builtin_fma(pe, o.er[b], accE_r[r][b]);
                        accE_i[r][b] = __builtin_fma(pe, o.ei[b], accE_i[r][b]);
                        accO_r[r][b] = __builtin_fma(po, o.orr[b], accO_r[r][b]);
                        accO_i[r][b] = __builtin_fma(po, o.oi[b], accO_i[r][b]);
                    }
                    const double Ae = __builtin_fma(z2h[r], o.be, o.abe);
                    const double Ao = __builtin_fma(z2h[r], o.bo, o.abo);
                    const double ne = __builtin_fma(Ae, p1[r][0].h, o.ge * pe);
                    const double no = __builtin_fma(Ao, p1[r][1].h, o.go * po);
                    p0[r][0].h = p1[r][0].h;
                    p1[r][0].h = ne;
                    p0[r][1].h = p1[r][1].h;
                    p1[r][1].h = no;
                }
            } else {
                const double *cle = cl + 4 * (2 * i + 2);
                const dd Be = {o.be, cle[0]}, ABe = {o.abe, cle[1]}, Ge = {o.ge, cle[2]};
                const dd Bo = {o.bo, cle[4]}, ABo = {o.abo, cle[5]}, Go = {o.go, cle[6]};
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const double pe = p0[r][0].h, po = p0[r][1].h;
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        accE_r[r][b] = __builtin_fma(pe, o.er[b], accE_r[r][b]);
                        accE_i[r][b] = __builtin_fma(pe, o.ei[b], accE_i[r][b]);
                        accO_r[r][b] = __builtin_fma(po, o.orr[b], accO_r[r][b]);
                        accO_i[r][b] = __builtin_fma(po, o.oi[b], accO_i[r][b]);
                    }
                    const dd z2 = {z2h[r], z2l[r]};
                    const dd Ae = dd_add(dd_mul(z2, Be), ABe);
                    const dd Ao = dd_add(dd_mul(z2, Bo), ABo);
                    const dd ne = dd_add(dd_mul(Ae, p1[r][0]), dd_mul(Ge, p0[r][0]));
                    const dd no = dd_add(dd_mul(Ao, p1[r][1]), dd_mul(Go, p0[r][1]));
                    p0[r][0] = p1[r][0];
                    p1[r][0] = ne;
                    p0[r][1] = p1[r][1];
                    p1[r][1] = no;
                }
            }
        };

        // chunks where both chains are inside l <= L
        const int c_full = (n1 / kChunk) * kChunk;
        int c = lo;
        for (; c < c_full; c += kChunk) {
            if (c <= hi) inject(c);
#pragma unroll
            for (int u = 0; u < kChunk; u++) compute(load_ops(c + u, true), c + u);
        }
        // tail: the odd chain may end first
        for (; c < n0; c += kChunk) {
            if (c <= hi) inject(c);
            for (int u = 0; u < kChunk; u++) {
                int i = c + u;
                if (i >= n0) break;
                compute(load_ops(i, i < n1), i);
            }
        }
    }

    // fused even/odd fold and store (Eqs. 13-14)
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (!gv[r] || k[r] >= a.n_north) continue;
        const int kn = k[r], ks = a.nrings - 1 - k[r];
        double *qn = a.q + 2 * (((size_t)kn * (a.L + 1) + m) * a.nmaps + a.map0);
        double *qs = a.q + 2 * (((size_t)ks * (a.L + 1) + m) * a.nmaps + a.map0);
#pragma unroll
        for (int b = 0; b < NB; b++) {
            double nr = accE_r[r][b] + accO_r[r][b], ni = accE_i[r][b] + accO_i[r][b];
            double sr = accE_r[r][b] - accO_r[r][b], si = accE_i[r][b] - accO_i[r][b];
            if (m == 0) ni = si = 0.0;  // real field: Im a_l0 is ignored
            *reinterpret_cast<double2 *>(qn + 2 * b) = make_double2(nr, ni);
            if (ks != kn) *reinterpret_cast<double2 *>(qs + 2 * b) = make_double2(sr, si);
        }
    }
}

// One launch covers every (m, ring block).  Workgroups are dispatched
// round-robin over the 8 XCDs: block b runs on XCD b % 8, and the ring
// blocks of one order m take consecutive slots of one XCD so that its L2
// serves the m's coefficient and a_lm stream to all of them.  Orders are
// visited from m = 0 (the longest chains) upward.  Within an order the
// compensated (double-double) waves nearest the poles come first, one 64-ring
// group each, so their long chains start early; they take the maps two at a
// time to stay inside the FP64 waves' register budget.  The FP64 waves
// follow with R groups each.
template <int NB, int R>
__global__ __launch_bounds__(64, (R == 4 ? 2 : 4)) void k_legendre(LegArgs a) {
    const int nrb = a.dd_groups + a.fp_blocks;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int m = 8 * (slot / nrb) + xcd;
    const int rb = slot % nrb;
    if (m > a.L) return;
    if (rb < a.dd_groups) {
        constexpr int NBD = NB < 2 ? NB : 2;
        for (int b0 = 0; b0 < NB; b0 += NBD) {
            LegArgs ab = a;
            ab.map0 = a.map0 + b0;
            legendre_wave<NBD, 1, true>(ab, m, rb);
        }
    } else {
        legendre_wave<NB, R, false>(a, m, a.dd_groups + (rb - a.dd_groups) * R);
    }
}

template <int NB, int R>
static hipError_t launch_nbr(const sht_plan_s *p, LegArgs a, hipStream_t st) {
    const int morders = (p->L + 1 + 7) / 8 * 8;  // orders rounded up to the XCD count
    a.dd_groups = p->n_dd_groups;
    a.fp_blocks = (a.ng - p->n_dd_groups + R - 1) / R;
    const long long grid = (long long)morders * (a.dd_groups + a.fp_blocks);
    hipLaunchKernelGGL((k_legendre<NB, R>), dim3((unsigned)grid), dim3(kLanes), 0, st, a);
    return hipGetLastError();
}

template <int NB>
static hipError_t launch_nb(const sht_plan_s *p, LegArgs a, hipStream_t st) {
    switch (p->rings_per_lane) {
        case 1: return launch_nbr<NB, 1>(p, a, st);
        case 4: return launch_nbr<NB, 4>(p, a, st);
        default: return launch_nbr<NB, 2>(p, a, st);
    }
}

// Persistent form for batches of requests (the many-transform regime of
// Sec. 3.4): one launch per wave shape (compensated waves of 2 or 1 maps,
// FP64 waves of 4, 2 or 1 maps) for every request of a batch, so that each
// launch runs one specialised body at its own occupancy.  Work items {pass,
// m, ring block, first map} of one shape come in eight lists, one per XCD
// (the items of one pass and order share a list, so that XCD's L2 serves the
// order's coefficient and a_lm stream to all of them), each sorted longest
// first and cut into chunks that shrink along the list.  A wave takes chunks
// from its own XCD's list through a device counter (a vector-memory atomic)
// and, once that list is exhausted, from the others in turn; it leaves when
// every counter has passed the end of its list, so every wave reaches the
// exit.  The wave body is k_legendre's.
constexpr int kQueueLists = 8;
constexpr int kQueueStride = 16;  // counters 64 bytes apart

__global__ void k_queue_reset(unsigned *c) {
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < kQueueShapes * kQueueLists; i += blockDim.x) c[i * kQueueStride] = 0u;
}

template <int NB, int R, bool DD>
__global__ __launch_bounds__(64, (R == 4 ? 2 : 4)) void k_legendre_queue(const LegArgs *__restrict__ passes,
                                                                         const int4 *__restrict__ items,
                                                                         const unsigned *__restrict__ chunk_off,
                                                                         const unsigned *__restrict__ list_off,
                                                                         unsigned *__restrict__ counter) {
    const int home = blockIdx.x & (kQueueLists - 1);  // workgroups are dealt to the XCDs round robin
    for (int s = 0; s < kQueueLists; s++) {
        const int x = (home + s) & (kQueueLists - 1);
        const unsigned lo = list_off[x], cnt = list_off[x + 1] - lo;
        for (;;) {
            unsigned c = 0;
            if (threadIdx.x == 0) c = atomicAdd(counter + x * kQueueStride, 1u);
            c = __shfl(c, 0);
            if (c >= cnt) break;
            const unsigned i0 = chunk_off[lo + c], i1 = chunk_off[lo + c + 1];
            for (unsigned i = i0; i < i1; i++) {
                const int4 w = items[i];
                const int pi = __builtin_amdgcn_readfirstlane(w.x), m = __builtin_amdgcn_readfirstlane(w.y);
                const int rb = __builtin_amdgcn_readfirstlane(w.z), b0 = __builtin_amdgcn_readfirstlane(w.w);
                LegArgs a = passes[pi];
                a.map0 += b0;
                if (DD)
                    legendre_wave<NB, 1, true>(a, m, rb);
                else
                    legendre_wave<NB, R, false>(a, m, a.dd_groups + (rb - a.dd_groups) * R);
            }
        }
    }
}

typedef void (*QueueKernel)(const LegArgs *, const int4 *, const unsigned *, const unsigned *, unsigned *);

template <int R>
static QueueKernel queue_kernel_r(int shape) {
    switch (shape) {
        case 0: return k_legendre_queue<2, 1, true>;
        case 1: return k_legendre_queue<1, 1, true>;
        case 2: return k_legendre_queue<4, R, false>;
        case 3: return k_legendre_queue<2, R, false>;
        default: return k_legendre_queue<1, R, false>;
    }
}

static QueueKernel queue_kernel(int shape, int R) {
    switch (R) {
        case 1: return queue_kernel_r<1>(shape);
        case 4: return queue_kernel_r<4>(shape);
        default: return queue_kernel_r<2>(shape);
    }
}

int queue_shape(bool dd, int nb) { return dd ? (nb >= 2 ? 0 : 1) : (nb >= 4 ? 2 : nb >= 2 ? 3 : 4); }

// Waves of the persistent launch of one shape: as many as the current device
// keeps resident at once.
hipError_t legendre_queue_grid(int shape, int rings_per_lane, int *grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)queue_kernel(shape, rings_per_lane), 64,
                                                         0);
    *grid = std::max(std::max(per_cu, 1) * std::max(cus, 1) / kQueueLists, 1) * kQueueLists;
    return e;
}

hipError_t launch_queue_reset(unsigned *counter, hipStream_t st) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, counter);
    return hipGetLastError();
}

hipError_t launch_legendre_queue(int shape, const LegArgs *passes, const int4 *items, const unsigned *chunk_off,
                                 const unsigned *list_off, unsigned *counter, int rings_per_lane, int grid,
                                 hipStream_t st) {
    if (shape < 0 || shape >= kQueueShapes || grid < 0) return hipErrorInvalidValue;
    if (grid == 0) return hipSuccess;  // no items of this shape
    hipLaunchKernelGGL(queue_kernel(shape, rings_per_lane), dim3((unsigned)grid), dim3(64), 0, st, passes, items,
                       chunk_off, list_off + shape * (kQueueLists + 1), counter + shape * kQueueLists * kQueueStride);
    return hipGetLastError();
}

// Argument block of one pass (maps map0 .. map0 + nb - 1 of nmaps) for
// waves of R rings per lane.
LegArgs leg_args(const sht_plan_s *p, int nmaps, int map0, int R, const double *alm, double *q) {
    LegArgs a;
    a.z2_hi = p->d_z2_hi;
    a.z2_lo = p->d_z2_lo;
    a.coef_off = p->d_coef_off;
    a.coef_hi = p->d_coef_hi;
    a.coef_lo = p->d_coef_lo;
    a.start_idx = p->d_start_idx;
    a.start_val = p->d_start_val;
    a.start_lo = p->d_start_lo;
    a.grp_lo = p->d_grp_lo;
    a.grp_hi = p->d_grp_hi;
    a.alm = alm;
    a.q = q;
    a.L = p->L;
    a.nrings = p->nrings;
    a.n_north = p->n_north;
    a.np = p->n_north_pad;
    a.n_dd_pad = std::max(p->n_dd_pad, 1);
    a.ng = p->n_north_pad / kLanes;
    a.nmaps = nmaps;
    a.map0 = map0;
    a.dd_groups = p->n_dd_groups;
    a.fp_blocks = (a.ng - p->n_dd_groups + R - 1) / R;
    return a;
}

hipError_t launch_legendre(const sht_plan_s *p, int nmaps, const double *alm, double *q,
                           hipStream_t stream) {
    LegArgs a;
    a.z2_hi = p->d_z2_hi;
    a.z2_lo = p->d_z2_lo;
    a.coef_off = p->d_coef_off;
    a.coef_hi = p->d_coef_hi;
    a.coef_lo = p->d_coef_lo;
    a.start_idx = p->d_start_idx;
    a.start_val = p->d_start_val;
    a.start_lo = p->d_start_lo;
    a.grp_lo = p->d_grp_lo;
    a.grp_hi = p->d_grp_hi;
    a.alm = alm;
    a.q = q;
    a.L = p->L;
    a.nrings = p->nrings;
    a.n_north = p->n_north;
    a.np = p->n_north_pad;
    a.n_dd_pad = std::max(p->n_dd_pad, 1);
    a.dd_groups = a.fp_blocks = 0;
    a.ng = p->n_north_pad / kLanes;
    a.nmaps = nmaps;
    hipError_t e = hipSuccess;
    // maps in passes of 4, then 2, then 1
    int b = 0;
    while (b < nmaps && e == hipSuccess) {
        a.map0 = b;
        int left = nmaps - b;
        if (left >= 4) {
            e = launch_nb<4>(p, a, stream);
            b += 4;
        } else if (left >= 2) {
            e = launch_nb<2>(p, a, stream);
            b += 2;
        } else {
            e = launch_nb<1>(p, a, stream);
            b += 1;
        }
    }
    return e;
}

}  // namespace sht
