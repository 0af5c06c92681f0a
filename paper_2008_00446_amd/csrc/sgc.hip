// The camera clustering {Phi_k} an LM iteration starts from, drawn on the
// device by stochastic graph clustering (Sec. 4.4, Eq. 16).
//
// The camera graph is the static block list of the Schur plan: block (r, c),
// r > c, holds one observation pair per point both cameras see, so its length
// is the edge weight w_rc.  From singletons, two neighbouring clusters whose
// joint size stays within gamma join with probability proportional to
// exp(beta dQ), dQ(x, y) = w_xy / s - K_x K_y / (2 s^2).  The draw uses
// competing exponential clocks: every eligible cluster pair (a, b), a < b (a
// cluster is named by its smallest camera), holds T = t_now + E / exp(beta dQ),
// E = -log u, u = ((x0 >> 11) + 1) 2^-53 from Philox4x64-10 with key (seed, 2)
// and counter (iteration, join step, a, b); the smallest clock (ties: smaller
// (a, b)) joins next, and only the pairs of the joined cluster get new clocks.
// This is the same law as drawing each join from Eq. 16's distribution.
//
// One 1024-thread workgroup runs the whole sequence of joins.  Thread t owns
// the pair slots of blocks t, t + 1024, ...; a slot keeps its pair's labels
// (a << 16 | b), its weight and its clock, in registers when the graph has at
// most 4096 blocks, else in the workspace.  Per join: (A) every
// slot that touches the joined clusters x, y is renamed to (x, z), and the
// slots of one neighbour z meet in LDS (smallest block index survives, weights
// summed with integer atomics); (B) survivors draw their new clock; the
// smallest clock is found by a wave reduction and one LDS round.  Two barriers
// per join.
#include "kernels.h"
#include "philox.h"

#include <limits.h>

namespace stba {
namespace {

constexpr int kSgcThreads = 1024;
constexpr int kSgcWaves = kSgcThreads / 64;
constexpr uint32_t kSgcDead = 0xFFFFFFFFu;
constexpr int kSgcRegSlots = 4;   // pair slots per thread kept in registers (graphs of <= 4096 blocks)
constexpr int kSgcBatch = 8;      // slots whose labels one round trip reads (larger graphs)
constexpr int kSgcAffList = 4;    // touched slots a thread remembers between the two phases (larger graphs)
constexpr int kSgcCompactEvery = 16;   // joins between two packings of the live slots (larger graphs)

// Per-camera state in dynamic LDS (24 bytes per camera, sgc_lds_bytes), the
// reductions in static LDS; the struct holds the pointers.
struct SgcSmall {
    double redT[kSgcWaves];
    uint32_t redP[kSgcWaves];
    int32_t redC[kSgcWaves];
    unsigned long long s_tot;
};
struct SgcShared {
    unsigned long long *K;   // summed incident weight of the cluster named i
    int32_t *lab;            // cluster name of each camera
    int32_t *csize;          // cameras in the cluster named i
    int32_t *slot;           // smallest block index of the renamed pairs (x, z), per z
    int32_t *wacc;           // their summed weight, per z; the cluster ranks at the end
    double *redT;
    uint32_t *redP;
    int32_t *redC;
    unsigned long long *s_tot;
};

__device__ inline bool clock_less(double t1, uint32_t p1, double t2, uint32_t p2) {
    return t1 < t2 || (t1 == t2 && p1 < p2);
}

// Clock of the pair (a, b) of weight w set at join step k, time t_now.
__device__ inline double pair_clock(int32_t a, int32_t b, int32_t w, unsigned long long Ka, unsigned long long Kb, double s,
                                    double beta, uint64_t seed, uint64_t iter, int32_t k, double t_now) {
#pragma clang fp contract(off)
    const uint64_t x0 = philox4x64_10_word0(iter, (uint64_t)k, (uint64_t)a, (uint64_t)b, seed, 2ull);
    const double u = (double)((x0 >> 11) + 1ull) * 0x1p-53;
    const double dq = (double)w / s - ((double)Ka * (double)Kb) / (2.0 * s * s);
    const double rate = exp(beta * dq);
    return t_now + (-log(u)) / rate;
}

// The smallest (clock, pair) over the workgroup, the same in every thread.
__device__ inline void block_argmin(double t, uint32_t p, SgcShared &sh, double &gt, uint32_t &gp) {
    for (int off = 32; off > 0; off >>= 1) {
        const double ot = __shfl_xor(t, off);
        const uint32_t op = (uint32_t)__shfl_xor((int)p, off);
        if (clock_less(ot, op, t, p)) {
            t = ot;
            p = op;
        }
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh.redT[wv] = t;
        sh.redP[wv] = p;
    }
    __syncthreads();
    gt = sh.redT[0];
    gp = sh.redP[0];
    for (int w = 1; w < kSgcWaves; ++w) {
        if (clock_less(sh.redT[w], sh.redP[w], gt, gp)) {
            gt = sh.redT[w];
            gp = sh.redP[w];
        }
    }
}

// The join sequence.  kRegs: at most S pair slots per thread, labels, weights
// and clocks in registers (loops unrolled); else any number of slots, all three
// in Pg / Wg / Tg (indexed by block, slot r of thread t is block 1024 r + t),
// the labels read kSgcBatch slots per round trip.
template <int S, bool kRegs>
__device__ void sgc_joins(int32_t m, int64_t nb, const int2 *blk_key, const int64_t *blk_start, int32_t gamma,
                          double beta, uint64_t seed, uint64_t iter, uint32_t *Pg, double *Tg, int32_t *Wg,
                          SgcShared &sh) {
    const int tid = threadIdx.x;
    const int nslots = (int)((nb + kSgcThreads - 1) / kSgcThreads);
    int nlive = nslots;   // larger graphs: this thread's slots in use, live ones packed to the front
    uint32_t Pr[kRegs ? S : 1];
    int32_t Wr[kRegs ? S : 1];
    double Tr[kRegs ? S : 1];
    auto gidx = [&](int r) { return r * kSgcThreads + tid; };
    auto wref = [&](int r) -> int32_t & { return kRegs ? Wr[kRegs ? r : 0] : Wg[gidx(r)]; };
    auto tref = [&](int r) -> double & { return kRegs ? Tr[kRegs ? r : 0] : Tg[gidx(r)]; };
    // f(r, P) -> the new label of the live slot r (P itself keeps it)
    auto for_live = [&](auto f) {
        if constexpr (kRegs) {
#pragma unroll
            for (int r = 0; r < S; ++r)
                if (Pr[r] != kSgcDead) Pr[r] = f(r, Pr[r]);
        } else {
            for (int r0 = 0; r0 < nlive; r0 += kSgcBatch) {
                uint32_t Pb[kSgcBatch];
#pragma unroll
                for (int j = 0; j < kSgcBatch; ++j) Pb[j] = r0 + j < nlive ? Pg[gidx(r0 + j)] : kSgcDead;
#pragma unroll
                for (int j = 0; j < kSgcBatch; ++j) {
                    if (Pb[j] == kSgcDead) continue;
                    const uint32_t Pn = f(r0 + j, Pb[j]);
                    if (Pn != Pb[j]) Pg[gidx(r0 + j)] = Pn;
                }
            }
        }
    };
    // the smallest (clock, label) over the live slots of this thread
    auto local_min = [&](double &tmin, uint32_t &pmin) {
        tmin = INFINITY;
        pmin = kSgcDead;
        if constexpr (kRegs) {
#pragma unroll
            for (int r = 0; r < S; ++r)
                if (Pr[r] != kSgcDead && clock_less(Tr[r], Pr[r], tmin, pmin)) {
                    tmin = Tr[r];
                    pmin = Pr[r];
                }
        } else {
            for (int r0 = 0; r0 < nlive; r0 += kSgcBatch) {
                uint32_t Pb[kSgcBatch];
                double Tb[kSgcBatch];
#pragma unroll
                for (int j = 0; j < kSgcBatch; ++j) Pb[j] = r0 + j < nlive ? Pg[gidx(r0 + j)] : kSgcDead;
#pragma unroll
                for (int j = 0; j < kSgcBatch; ++j) Tb[j] = Pb[j] != kSgcDead ? Tg[gidx(r0 + j)] : INFINITY;
#pragma unroll
                for (int j = 0; j < kSgcBatch; ++j)
                    if (Pb[j] != kSgcDead && clock_less(Tb[j], Pb[j], tmin, pmin)) {
                        tmin = Tb[j];
                        pmin = Pb[j];
                    }
            }
        }
    };

    long long my_s = 0;
    for (int r = 0; r < (kRegs ? S : nslots); ++r) {
        const int64_t b = (int64_t)r * kSgcThreads + tid;
        uint32_t P = kSgcDead;
        if (b < nb) {
            const int2 key = blk_key[b];
            if (key.x != key.y) {
                const int32_t w = (int32_t)(blk_start[b + 1] - blk_start[b]);
                P = ((uint32_t)key.y << 16) | (uint32_t)key.x;   // (c, r): c < r
                wref(r) = w;
                atomicAdd(&sh.K[key.y], (unsigned long long)w);
                atomicAdd(&sh.K[key.x], (unsigned long long)w);
                my_s += w;
            }
        }
        if constexpr (kRegs)
            Pr[kRegs ? r : 0] = P;
        else
            Pg[gidx(r)] = P;
    }
    for (int off = 32; off > 0; off >>= 1) my_s += __shfl_xor(my_s, off);
    if ((tid & 63) == 0 && my_s) atomicAdd(sh.s_tot, (unsigned long long)my_s);
    __syncthreads();
    const double s = (double)*sh.s_tot;
    const bool any = s > 0.0 && gamma > 1;

    // initial clocks (join step 0, time 0)
    for_live([&](int r, uint32_t P) -> uint32_t {
        if (!any) return kSgcDead;
        const int32_t a = (int32_t)(P >> 16), b = (int32_t)(P & 0xFFFFu);
        tref(r) = pair_clock(a, b, wref(r), sh.K[a], sh.K[b], s, beta, seed, iter, 0, 0.0);
        return P;
    });
    double tmin, gt;
    uint32_t pmin, gp;
    local_min(tmin, pmin);
    block_argmin(tmin, pmin, sh, gt, gp);

    for (int32_t k = 1; k < m && gt < INFINITY; ++k) {
        const int32_t x = (int32_t)(gp >> 16), y = (int32_t)(gp & 0xFFFFu);
        const double t_now = gt;
        if (!kRegs && (k & (kSgcCompactEvery - 1)) == 0) {
            // pack this thread's live slots to the front (label, weight and clock move together)
            int w = 0;
            for (int r0 = 0; r0 < nlive; r0 += kSgcBatch) {
                uint32_t Pb[kSgcBatch];
#pragma unroll
                for (int j = 0; j < kSgcBatch; ++j) Pb[j] = r0 + j < nlive ? Pg[gidx(r0 + j)] : kSgcDead;
#pragma unroll
                for (int j = 0; j < kSgcBatch; ++j) {
                    if (Pb[j] == kSgcDead) continue;
                    if (w != r0 + j) {
                        Pg[gidx(w)] = Pb[j];
                        Wg[gidx(w)] = Wg[gidx(r0 + j)];
                        Tg[gidx(w)] = Tg[gidx(r0 + j)];
                    }
                    ++w;
                }
            }
            nlive = w;
        }
        // (A) join y into x; the pairs of x and y meet per neighbour z
        if (tid == 0) {
            sh.csize[x] += sh.csize[y];
            sh.K[x] += sh.K[y];
        }
        for (int32_t i = tid; i < m; i += kSgcThreads)
            if (sh.lab[i] == y) sh.lab[i] = x;
        bool rescan = pmin == gp;
        // the slots of this thread that touch x or y (the first kSgcAffList of them)
        int naff = 0;
        int affr[kSgcAffList];
        for_live([&](int r, uint32_t P) -> uint32_t {
            if (P == gp) return kSgcDead;
            const int32_t a = (int32_t)(P >> 16), b = (int32_t)(P & 0xFFFFu);
            if (a == x || a == y || b == x || b == y) {
                const int32_t z = (a == x || a == y) ? b : a;
                rescan |= P == pmin;
                atomicMin(&sh.slot[z], gidx(r));
                atomicAdd(&sh.wacc[z], wref(r));
                if (!kRegs) {
#pragma unroll
                    for (int i = 0; i < kSgcAffList; ++i)
                        if (naff == i) affr[i] = r;
                    ++naff;
                }
            }
            return P;
        });
        __syncthreads();
        // (B) one survivor per neighbour takes the summed weight and a new clock
        bool fresh = false;
        double fT = INFINITY;
        uint32_t fP = kSgcDead;
        auto survive = [&](int r, uint32_t P) -> uint32_t {
            const int32_t a = (int32_t)(P >> 16), b = (int32_t)(P & 0xFFFFu);
            if (!(a == x || a == y || b == x || b == y)) return P;
            const int32_t z = (a == x || a == y) ? b : a;
            if (sh.slot[z] != gidx(r)) return kSgcDead;
            const int32_t w = sh.wacc[z];
            sh.slot[z] = INT_MAX;
            sh.wacc[z] = 0;
            if (sh.csize[x] + sh.csize[z] > gamma) return kSgcDead;
            const int32_t lo = x < z ? x : z, hi = x < z ? z : x;
            const uint32_t Pn = ((uint32_t)lo << 16) | (uint32_t)hi;
            const double T = pair_clock(lo, hi, w, sh.K[lo], sh.K[hi], s, beta, seed, iter, k, t_now);
            wref(r) = w;
            tref(r) = T;
            fresh = true;
            if (clock_less(T, Pn, fT, fP)) {
                fT = T;
                fP = Pn;
            }
            return Pn;
        };
        if (kRegs || naff > kSgcAffList) {
            for_live(survive);
        } else {
#pragma unroll
            for (int i = 0; i < kSgcAffList; ++i) {
                if (i < naff) {
                    const int r = affr[i];
                    const uint32_t P = Pg[gidx(r)];
                    const uint32_t Pn = survive(r, P);
                    if (Pn != P) Pg[gidx(r)] = Pn;
                }
            }
        }
        if (rescan)
            local_min(tmin, pmin);
        else if (fresh && clock_less(fT, fP, tmin, pmin)) {
            tmin = fT;
            pmin = fP;
        }
        block_argmin(tmin, pmin, sh, gt, gp);
    }
}

__global__ __launch_bounds__(kSgcThreads) void k_sgc(int32_t m, const int64_t *n_blocks, const int2 *blk_key,
                                                     const int64_t *blk_start, int32_t gamma, double beta,
                                                     uint64_t seed, uint64_t iter, uint32_t *Pg, double *Tg,
                                                     int32_t *Wg, int32_t *cam_cluster, int32_t *n_clusters,
                                                     int32_t *status) {
    extern __shared__ __align__(16) unsigned long long sgc_lds[];
    __shared__ SgcSmall small;
    SgcShared sh;
    sh.K = sgc_lds;
    sh.lab = reinterpret_cast<int32_t *>(sgc_lds + m);
    sh.csize = sh.lab + m;
    sh.slot = sh.csize + m;
    sh.wacc = sh.slot + m;
    sh.redT = small.redT;
    sh.redP = small.redP;
    sh.redC = small.redC;
    sh.s_tot = &small.s_tot;
    const int tid = threadIdx.x;
    const int64_t nb = n_blocks[0];
    for (int32_t i = tid; i < m; i += kSgcThreads) {
        sh.lab[i] = i;
        sh.csize[i] = 1;
        sh.slot[i] = INT_MAX;
        sh.wacc[i] = 0;
        sh.K[i] = 0;
    }
    if (tid == 0) *sh.s_tot = 0;
    __syncthreads();
    if (nb <= kSgcRegSlots * kSgcThreads)
        sgc_joins<kSgcRegSlots, true>(m, nb, blk_key, blk_start, gamma, beta, seed, iter, Pg, Tg, Wg, sh);
    else
        sgc_joins<1, false>(m, nb, blk_key, blk_start, gamma, beta, seed, iter, Pg, Tg, Wg, sh);
    __syncthreads();

    // number the clusters 0..l-1 by their smallest camera (= their name): the
    // rank of each name among the names, by a block scan over camera ranges
    constexpr int kPer = kSgcMaxCams / kSgcThreads;
    int32_t cnt = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int32_t i = tid * kPer + j;
        if (i < m && sh.lab[i] == i) ++cnt;
    }
    int32_t incl = cnt;
    const int lane = tid & 63;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    if (lane == 63) sh.redC[tid >> 6] = incl;
    __syncthreads();
    int32_t base = incl - cnt;
    int32_t total = 0;
    for (int w = 0; w < kSgcWaves; ++w) {
        if (w < (tid >> 6)) base += sh.redC[w];
        total += sh.redC[w];
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int32_t i = tid * kPer + j;
        if (i < m && sh.lab[i] == i) sh.wacc[i] = base++;
    }
    __syncthreads();
    for (int32_t i = tid; i < m; i += kSgcThreads) cam_cluster[i] = sh.wacc[sh.lab[i]];
    if (tid == 0) {
        *n_clusters = total;
        *status = STBA_OK;
    }
}

}  // namespace

hipError_t launch_sgc(int32_t m, const int64_t *n_blocks, const int2 *blk_key, const int64_t *blk_start,
                      int32_t gamma, double beta, uint64_t seed, uint64_t iter, uint32_t *Pg, double *Tg,
                      int32_t *Wg, int32_t *cam_cluster, int32_t *n_clusters, int32_t *status, hipStream_t st) {
    // 8 bytes of K and 4 x 4 of the int32 arrays per camera
    const size_t lds = 24 * (size_t)m;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_sgc),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_sgc<<<1, kSgcThreads, lds, st>>>(m, n_blocks, blk_key, blk_start, gamma, beta, seed, iter, Pg, Tg, Wg,
                                       cam_cluster, n_clusters, status);
    return hipGetLastError();
}

}  // namespace stba
