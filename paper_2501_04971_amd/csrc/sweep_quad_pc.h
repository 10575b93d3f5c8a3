// Producer/consumer form of the quadratic annealing run, for launches that
// leave SIMDs idle (one wave of 64 replicas per CU): a workgroup is one
// consumer wave that walks the sites of its 64 replicas, plus six (two per
// SIMD, the default) or three producer waves on the CU's other SIMDs that do the part of
// every visit that does not depend on the state, one block of 32 sites ahead:
//
//  * the Philox4x32-10 draw u24 of the visit (same counters as everywhere);
//  * its threshold index j* = min{ j : Theta[j] > u24 } (Theta is
//    non-decreasing, so x_i = [u24 < Theta[idx]] = [idx >= j*]), from the
//    inverse of tanh checked against one adjacent pair of table entries (a
//    third entry for guesses one position off, an exact bisection for the
//    rare draws in the table's flat tails);
//  * the threshold on the field itself: with
//      hi = floor((Z B_t + 2^(S'-1)) / 2^32),  idx = clamp(floor(hi / 2^ish)),
//    and -2304 < j* <= 2304, [idx >= j*] = [hi >= j* 2^ish] = [Z >= Zt] with
//    Zt = ceil((2 j* - 1) 2^(ish+31) / B_t) (field_threshold: exact, from
//    per-sweep constants);
//  * the refill of the J slab two blocks ahead.
//
// The consumer's visit is then the field and one 64-bit compare; the per-site thresholds arrive through a double-buffered LDS ring
// (32 sites x 64 lanes x 8 bytes per block) and one workgroup barrier per
// block hands buffers over.  The consumer also issues the next block's field
// refresh on the matrix cores while it visits the current block (see
// NextFields).  Results are bit-identical to sweep_quad.
#pragma once
#include "sweep_quad.h"

namespace pbit {

// The threshold table of the split quadratic kernel is stored as pairs:
// 8-byte entry k holds Theta[k] and Theta[k + 1], so that a producer's probe
// of two adjacent entries is one aligned 64-bit read.
constexpr int kThetaPairBytes = kThetaLen * 8 + 8;  // rounded up to 16 bytes

template <int NB>
constexpr size_t quad_pc_lds_bytes()
{
    return (size_t)kThetaPairBytes + (size_t)NB * 32 * 32 + 3 * (size_t)1024 * (NB + 1) + kRingBytes;
}

// Operands of one consumer visit, read from LDS a few visits ahead so that
// the read latency stays off the chain of decisions: the threshold from the
// ring, the record constant for the site's block-start state, the weight, and
// the site's row of the strictly lower in-block part of W.
struct VisitOps {
    int64_t thr, K;
    int32_t meta;
    uint32_t w[8];
};

template <int s, int LS>
__device__ __forceinline__ void load_visit_ops(VisitOps &o, const BlockVisit &v, const uint32_t (&x0)[8],
                                               const int64_t *ring)
{
    if constexpr (s < 32) {
        // site s changes only at its own visit, so its old state is known from
        // the block-start copy and the record is indexed by it
        const uint32_t xo = (x0[s >> 2] >> (8 * (s & 3))) & 1u;
        const int64_t *cur = v.rec + 4 * s;
        o.thr = ring[s * 64 + (threadIdx.x & 63)];
        o.K = cur[xo];
        o.meta = *reinterpret_cast<const int32_t *>(cur + 3);
        const uint32_t *wrow = reinterpret_cast<const uint32_t *>(v.wblk + s * LS);
#pragma unroll
        for (int w = 0; w < (s + 3) / 4; ++w) o.w[w] = wrow[w];
    }
}

// Consumer visit of site s: the ring holds the threshold on the field itself,
// or, with parallel tempering (every lane at the temperature of its ladder
// position, which the producers do not know), the draw's table position j*,
// which the visit compares with the index of its own field: [idx >= j*] is
// the update [u24 < Theta[idx]].  The replica's energy follows every flip.
template <int s, bool PT = false>
__device__ __forceinline__ void visit_site_pc(BlockVisit &v, uint32_t (&xc)[8], const uint32_t (&x0)[8],
                                              const VisitOps &o)
{
    const uint32_t xo = (x0[s >> 2] >> (8 * (s & 3))) & 1u;
    // block-start field plus the block's earlier sites at their current states
    int32_t f = v.F[s];
#pragma unroll
    for (int w = 0; w < (s + 3) / 4; ++w) f = __builtin_amdgcn_sdot4((int)o.w[w], (int)xc[w], f, false);
    // v.k2 holds -k2 here
    const int64_t Z = o.K + (int64_t)(f * 256) * v.sg2 + (int64_t)__mul24(o.meta, v.g) * v.k2;
    uint32_t xn;
    if constexpr (PT)  // (sites beyond N_ext hold INT64_MAX: never on)
        xn = (int64_t)theta_index(Z, v.Bt, v.ish, v.irnd, v.hclo, v.hchi) >= o.thr ? 1u : 0u;
    else
        xn = Z >= o.thr ? 1u : 0u;
    const int32_t delta = (int32_t)xn - (int32_t)xo;
    xc[s >> 2] += (uint32_t)delta << (8 * (s & 3));
    v.g += __mul24(delta, o.meta);
    if constexpr (PT) v.E = delta > 0 ? v.E - Z : (delta < 0 ? v.E + Z : v.E);
}

// Fields of the next block, accumulated on the matrix cores while the current
// block is visited.  With the state rotated so that x[0] is the current block
// b, the next block's field is W[b+1, :] . x = sum over chunks p = 1 .. NB-1 of
// W[b+1, chunk (b+p)] . x[p] (unchanged by this block's visits; p = 1 is the
// next block's own chunk, without its strictly lower part) plus
// W[b+1, chunk b] . x[0], added once the visits are done.  The partial products
// are spread over the visits (one MFMA pair every STEP visits, operands loaded
// at the block start), so their latency overlaps the visit chain instead of
// adding to it.
template <int NB>
struct NextFields {
    v16i acc0, acc1;
    const int8_t *arow;             // LDS: this lane's A-operand row of the next block's slab
    const int8_t *adiag;            // LDS: its A operand of that slab's diagonal chunk (diag_arow)
    v4i a[NB > 1 ? NB - 1 : 1];     // A operands of chunks p = 1 .. NB-1, loaded at the block start

    // x[p] holds block (b + p) mod NB, whose columns of the next block's rows
    // are chunk (b + p) mod NB of the slab
    __device__ __forceinline__ void load(int b)
    {
#pragma unroll
        for (int p = 1; p < NB; ++p) {
            int c = b + p;
            c = c >= NB ? c - NB : c;
            a[p - 1] = *reinterpret_cast<const v4i *>(p == 1 ? adiag : arow + c * 32);
        }
    }
};

template <int s, int NB>
__device__ __forceinline__ void next_fields_step(NextFields<NB> &nf, const uint32_t (&x)[NB][8])
{
    constexpr int STEP = NB > 1 ? 32 / (NB - 1) : 33;
    if constexpr (NB > 1 && s % STEP == 0 && s / STEP < NB - 1) {
        constexpr int p = s / STEP + 1;
        const v4i A = nf.a[p - 1];
        const v4i B0 = {(int)x[p][0], (int)x[p][1], (int)x[p][2], (int)x[p][3]};
        const v4i B1 = {(int)x[p][4], (int)x[p][5], (int)x[p][6], (int)x[p][7]};
        nf.acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B0, nf.acc0, 0, 0, 0);
        nf.acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B1, nf.acc1, 0, 0, 0);
    }
}

// Scheduling window of the visiting wave (see visit_fence) and how many
// visits ahead it reads its operands.
#ifndef PBIT_PC_SCHED_WINDOW
#define PBIT_PC_SCHED_WINDOW 4
#endif
#ifndef PBIT_PC_PREFETCH
#define PBIT_PC_PREFETCH 4
#endif

template <int LS, int NB, bool PT, int... S>
__device__ __forceinline__ void visit_block_pc(BlockVisit &v, uint32_t (&x)[NB][8], NextFields<NB> &nf,
                                               const int64_t *ring, std::integer_sequence<int, S...>)
{
    constexpr int PF = PBIT_PC_PREFETCH;
    const uint32_t x0[8] = {x[0][0], x[0][1], x[0][2], x[0][3], x[0][4], x[0][5], x[0][6], x[0][7]};
    VisitOps ops[PF];
    // the operands of the first PF visits, then each visit reads those of the
    // visit PF places later into the slot it has just used
    ((S < PF ? load_visit_ops<S < PF ? S : 32, LS>(ops[S % PF], v, x0, ring) : void()), ...);
    ((visit_site_pc<S, PT>(v, x[0], x0, ops[S % PF]), load_visit_ops<S + PF, LS>(ops[S % PF], v, x0, ring),
      next_fields_step<S, NB>(nf, x), visit_fence<S, PBIT_PC_SCHED_WINDOW>()),
     ...);
}

// Guess of the largest table position p with th[p] <= u from the inverse of
// the generating function 2^24 (1 + tanh(j/256))/2 at u + 1/2 (hardware log2),
// clamped so that p - 1 .. p + 2 are table positions; the caller checks it.
__device__ __forceinline__ int theta_floor_guess(uint32_t u)
{
    const float v = (float)u + 0.5f;
    const float j = 88.72283911167299f * (__log2f(v) - __log2f(16777216.0f - v));  // 128 ln 2 = 88.72...
    const int p = (int)floorf(j) + kThetaHalf;
    return min(max(p, 1), kThetaLen - 3);
}

// Producer p (0 .. NP-1 of NP = 3 or 6) fills its share of the ring buffer of
// block blk (sites 32 blk .. 32 blk + 31) of sweep t: Philox groups g = p + NP k
// (four sites each), k < KG.  The KG groups run side by side with no branch
// between the table searches, so the scheduler can overlap them.  The
// table position of each draw comes from theta_floor_guess, accepted only where
// the table confirms it: one pair read settles all but about one draw in 10^4,
// a third entry those one position off, and an exact bisection over the whole
// table the rest (flat tails, where many positions share a value: a few draws
// in 10^6).  Sites at or beyond N_ext never flip.
// PAIR: th is the pair table (entry k at th[2k], th[2k + 1] = Theta[k + 1]).
template <int NP, int KG, bool JSTAR, bool PAIR>
__device__ __forceinline__ void produce_groups(const DevInstance &d, int p, int t, int blk, int64_t *ring,
                                               const int32_t *th, uint32_t kround, uint64_t m2)
{
    auto entry = [th](int k) { return (uint32_t)th[PAIR ? 2 * k : k]; };
    constexpr int E = 4 * KG;
    const int lane = threadIdx.x & 63;
    const uint32_t cbase = (uint32_t)t * (uint32_t)d.nq;
    uint32_t u[E];
    int gs[E];
#pragma unroll
    for (int k = 0; k < KG; ++k) {
        uint32_t rnd[4];
        philox_block(cbase + (uint32_t)(blk * 8 + p + NP * k), kround, m2, d.inst_id, d.seed_lo, d.seed_hi, rnd);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u[4 * k + q] = rnd[q] >> 8;
            gs[4 * k + q] = theta_floor_guess(u[4 * k + q]);
        }
    }
    int lo[E], hi[E];
    int dir[E];
    bool miss = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        // fast path: one read of the adjacent pair th[g], th[g + 1] settles the
        // draw when th[g] <= u < th[g + 1] (position g); otherwise dir says on
        // which side the position lies (th is non-decreasing)
        const int g = gs[e];
        uint32_t t1, t2;
        if constexpr (PAIR) {
            const uint2 pr = *reinterpret_cast<const uint2 *>(th + 2 * g);
            t1 = pr.x;
            t2 = pr.y;
        } else {
            t1 = (uint32_t)th[g];
            t2 = (uint32_t)th[g + 1];
        }
        const bool skip = p + NP * (e >> 2) >= 8;  // a discarded group needs no search
        dir[e] = skip ? 0 : (t1 > u[e] ? -1 : (t2 <= u[e] ? 1 : 0));
        lo[e] = g;
        hi[e] = g;
        miss = miss || dir[e] != 0;
    }
    // second chance for the draws whose guess is one position off (about one
    // draw in 10^4, so a wave takes this branch for a minority of blocks): the
    // entry beyond the pair confirms position g - 1 or g + 1; anything further
    // off (the flat tails of the table) goes to the bisection below
    if (__ballot(miss)) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (dir[e] != 0) {
                const int g = gs[e];
                const uint32_t t3 = entry(dir[e] < 0 ? g - 1 : g + 2);
                const bool ok = dir[e] < 0 ? t3 <= u[e] : u[e] < t3;
                lo[e] = ok ? g + dir[e] : 0;
                hi[e] = ok ? g + dir[e] : kThetaLen - 1;
            }
        }
    }
    // exact bisection for the draws the fast path did not settle: th[lo] <= u
    // holds throughout (th[0] = 0), and the search ends at the largest such lo
    for (;;) {
        bool any = false;
#pragma unroll
        for (int e = 0; e < E; ++e) any = any || lo[e] < hi[e];
        if (__ballot(any) == 0) break;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (lo[e] < hi[e]) {
                const int mid = (lo[e] + hi[e] + 1) >> 1;
                const bool le = entry(mid) <= u[e];
                lo[e] = le ? mid : lo[e];
                hi[e] = le ? hi[e] : mid - 1;
            }
        }
    }
    // Thresholds on the carried field, Zt = ceil((2 j* - 1) 2^E / B_t), exact,
    // from the sweep's constants (a uniform load).  Nearly every sweep takes
    // the short form; a draw whose estimate lies next to an integer (about one
    // in 10^9) makes its wave redo that draw exactly.  The thresholds are
    // stored after all of them are known (stores between the computations
    // made the whole kernel a third slower, measured).
    int64_t h[E];
    if constexpr (JSTAR) {
        // parallel tempering: the table position itself
#pragma unroll
        for (int e = 0; e < E; ++e) h[e] = lo[e] + 1 - kThetaHalf;
    } else {
    const ZtSweep zs = d.zsweep[t];
    if (zs.fast) {
        bool near[E], any = false;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            h[e] = field_threshold_fast(2 * (lo[e] + 1 - kThetaHalf) - 1, zs, &near[e]);
            any = any || near[e];
        }
        if (__ballot(any)) {
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (near[e]) h[e] = field_threshold(2 * (lo[e] + 1 - kThetaHalf) - 1, zs);
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) h[e] = field_threshold(2 * (lo[e] + 1 - kThetaHalf) - 1, zs);
    }
    }
#pragma unroll
    for (int k = 0; k < KG; ++k) {
        if (p + NP * k < 8) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int s = 4 * (p + NP * k) + q;
                ring[s * 64 + lane] = blk * 32 + s < d.n_ext ? h[4 * k + q] : INT64_MAX;
            }
        }
    }
}

// Producer p owns the Philox groups p, p + NP, p + 2 NP, ... below 8: the first
// 8 - NP (KMAX - 1) producers take KMAX of them, the others one fewer (with
// NP = 6, two per SIMD, the SIMDs then carry 3, 3 and 2 groups).
template <int NP, bool JSTAR = false, bool PAIR = false>
__device__ __forceinline__ void produce_thresholds(const DevInstance &d, int p, int t, int blk, int64_t *ring,
                                                   const int32_t *th, uint32_t kround, uint64_t m2)
{
    constexpr int KMAX = (8 + NP - 1) / NP;
    if (p + NP * (KMAX - 1) < 8)
        produce_groups<NP, KMAX, JSTAR, PAIR>(d, p, t, blk, ring, th, kround, m2);
    else
        produce_groups<NP, KMAX - 1, JSTAR, PAIR>(d, p, t, blk, ring, th, kround, m2);
}

// Producer p's share of the next J slab (quadratic kernel): loaded into
// registers before the producer's other work of the block and stored after
// it, so that the global loads' latency is hidden.
template <int NB, int NP>
constexpr int slab_pieces_per_producer()
{
    return (NB + 1 + NP - 1) / NP;
}

template <int NB, int NP>
__device__ __forceinline__ void load_slab(int p, const int8_t *jsrc, uint4 (&pf)[slab_pieces_per_producer<NB, NP>()])
{
    constexpr int PIECES = NB + 1;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < slab_pieces_per_producer<NB, NP>(); ++j)
        pf[j] = *reinterpret_cast<const uint4 *>(jsrc + min(p + NP * j, PIECES - 1) * 1024 + lane * 16);
}

template <int NB, int NP>
__device__ __forceinline__ void store_slab(int p, int8_t *ldst, const uint4 (&pf)[slab_pieces_per_producer<NB, NP>()])
{
    constexpr int PIECES = NB + 1;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < slab_pieces_per_producer<NB, NP>(); ++j)
        *reinterpret_cast<uint4 *>(ldst + min(p + NP * j, PIECES - 1) * 1024 + lane * 16) = pf[j];
}

// Waves of the split workgroup for PR producers: wave 0 visits; with PR = 3
// waves 1-3 produce; with PR = 6 waves 1-3 and 5-7 produce and wave 4 (which
// shares the visiting wave's SIMD, waves being placed round-robin) only takes
// part in the barriers.
template <int PR>
constexpr int quad_pc_waves()
{
    return PR == 3 ? 4 : 8;
}

// One annealing run of replicas rbase + [0, 64) by a workgroup of
// quad_pc_waves<PR>() waves, then the scoring of the final states.  smem must
// hold quad_pc_lds_bytes<NB>() bytes.
template <int NB, int PR, bool PT = false>
__device__ __forceinline__ void quad_run_pc(const DevInstance &d, int rbase, unsigned char *smem)
{
    static_assert(PR == 3 || PR == 6, "3 or 6 producers");
    constexpr int NP = NB * 32;
    constexpr int LS = NP + 16;
    constexpr int SLAB = 1024 * (NB + 1);
    int32_t *th = reinterpret_cast<int32_t *>(smem);  // pair table
    int64_t *site = reinterpret_cast<int64_t *>(smem + kThetaPairBytes);
    int8_t *slabs = reinterpret_cast<int8_t *>(smem + kThetaPairBytes + NP * 32);  // three buffers
    int64_t *ring = reinterpret_cast<int64_t *>(smem + kThetaPairBytes + NP * 32 + 3 * SLAB);

    // the slab of block step c (block c % NB) sits in buffer c % 3 during steps
    // c - 1 (the next block's fields) and c (its in-block couplings)
    copy_slab<NB>(d.J, 0, slabs);
    copy_slab<NB>(d.J, 1 % NB, slabs + SLAB);
    for (int e = threadIdx.x; e < kThetaLen; e += blockDim.x) {
        th[2 * e] = d.theta[e];
        th[2 * e + 1] = d.theta[e + 1 < kThetaLen ? e + 1 : e];
    }
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(d.site);
        uint4 *dst = reinterpret_cast<uint4 *>(site);
        for (int e = threadIdx.x; e < NP * 2; e += blockDim.x) dst[e] = src[e];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    // wave-uniform by construction; saying so lets the compiler split consumer
    // and producers with scalar branches
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int r = rbase + lane;  // every wave serves the same 64 replicas
    const uint32_t kround = (uint32_t)d.round_k[0];
    const uint64_t m2 = (uint64_t)0xCD9E8D57u * (uint32_t)r;
    const int total = d.T * NB;

    const bool producer = wave > 0 && !(PR == 6 && wave == 4);
    const int pi = PR == 6 && wave > 4 ? wave - 2 : wave - 1;  // producer index 0 .. PR-1
    if (producer) produce_thresholds<PR, PT, true>(d, pi, 0, 0, ring, th, kround, m2);
    __syncthreads();

    uint32_t x[NB][8];
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
        for (int w = 0; w < 8; ++w) x[p][w] = 0u;

    BlockVisit v;
    v.th = th;
    v.g = -(int32_t)d.b[0];
    v.ish = d.ish;
    v.hclo = d.hclo;
    v.hchi = d.hchi;
    v.irnd = d.irnd;
    v.sg2 = d.sg2;
    v.k2 = (int64_t)(int32_t)(-d.k2);  // 0 <= k2 < 2^31, so -k2 is an int32
    v.kround = kround;
    v.inst = d.inst_id;
    v.seed_lo = d.seed_lo;
    v.seed_hi = d.seed_hi;
    v.m2 = m2;
    v.wave = wave;
    v.nw = 1;
    // parallel tempering: the replica's ladder position, the lane this lane
    // keeps track of (the one at position lane mod L), the replica's energy
    int32_t slot = 0, owner = lane;
    v.E = 0;
    v.Bt = 0;
    if constexpr (PT) slot = lane & (d.pt - 1);

    if (wave == 0) block_fields<NB>(slabs, 0, x, v.F);  // fields of the first block

    int buf = 0;         // ring buffer of block step c
    int b0 = 0, b1 = 1;  // slab buffers of steps c and c + 1 (c % 3, (c + 1) % 3)
    for (int c = 0; c < total; ++c) {
        const int blk = c - (c / NB) * NB;
        const int b2 = b1 == 2 ? 0 : b1 + 1;
        if (wave == 0) {
            const int8_t *slab = slabs + b0 * SLAB;
#pragma unroll
            for (int w = 0; w < 4; ++w) swap_halves(x[0][w], x[0][w + 4]);
            v.rec = site + 4 * (blk * 32);
            v.wblk = slab + blk * 32;
            v.blk = blk;
            NextFields<NB> nf;
            nf.acc0 = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            nf.acc1 = nf.acc0;
            nf.arow = slabs + b1 * SLAB + (lane & 31) * LS + (lane >> 5) * 16;
            nf.adiag = diag_arow<NB>(slabs + b1 * SLAB, lane);
            nf.load(blk);
            if (PT && blk == 0) v.Bt = d.bladder[slot];  // this sweep's temperature
            visit_block_pc<LS, NB, PT>(v, x, nf, ring + buf * 32 * 64, std::make_integer_sequence<int, 32>{});
#pragma unroll
            for (int w = 0; w < 4; ++w) swap_halves(x[0][w], x[0][w + 4]);
            {
                // this block's chunk completes the next block's fields (with one
                // block the next block is this one again: its diagonal chunk)
                const v4i A = *reinterpret_cast<const v4i *>(NB == 1 ? nf.adiag : nf.arow + blk * 32);
                const v4i B0 = {(int)x[0][0], (int)x[0][1], (int)x[0][2], (int)x[0][3]};
                const v4i B1 = {(int)x[0][4], (int)x[0][5], (int)x[0][6], (int)x[0][7]};
                nf.acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B0, nf.acc0, 0, 0, 0);
                nf.acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B1, nf.acc1, 0, 0, 0);
            }
            rotate_chunks<NB>(x);
            fields_from_acc(nf.acc0, nf.acc1, v.F);
            if (PT && blk == NB - 1) pt_exchange(d, c / NB, kround, m2, v.E, owner, slot);  // after each sweep
        } else if (producer) {
            // the next block's thresholds, and the slab of the block after it
            // (at the end: slabs 0 and 1 for the scoring pass, no thresholds)
            const int t1 = (c + 1) / NB, blk1 = (c + 1) - t1 * NB;
            const int blk2 = (c + 2) % NB;
            uint4 pf[slab_pieces_per_producer<NB, PR>()];
            load_slab<NB, PR>(pi, d.J + (size_t)blk2 * SLAB, pf);
            if (c + 1 < total)
                produce_thresholds<PR, PT, true>(d, pi, t1, blk1, ring + (buf ^ 1) * 32 * 64, th, kround, m2);
            store_slab<NB, PR>(pi, slabs + b2 * SLAB, pf);
        }
        buf ^= 1;
        b0 = b1;
        b1 = b2;
        __syncthreads();
    }

    // score the final state (wave 0); all waves help refill the slabs
    const int n = d.n, n_ext = d.n_ext;
    const bool live = wave == 0 && r < d.R;
    int64_t pacc = 0;
    int32_t sval = 0;
    // slab 0 is in buffer b0 after the last block wrapped around (and slab 1 in b1)
    for (int blk = 0; blk < NB; ++blk) {
        const int8_t *slab = slabs + b0 * SLAB;
        if (blk + 1 < NB) copy_slab<NB>(d.J, blk + 1, slabs + b1 * SLAB);
        if (wave == 0) {
            int32_t F[32];
            block_fields<NB, true>(slab, blk, x, F);
#pragma unroll
            for (int w = 0; w < 4; ++w) swap_halves(x[0][w], x[0][w + 4]);
            uint32_t bits = 0;
#pragma unroll
            for (int w = 0; w < 8; ++w) bits |= bytes_to_nibble(x[0][w]) << (4 * w);
            if (live && blk < d.words) d.rx[(int64_t)r * d.words + blk] = bits;
#pragma unroll
            for (int s = 0; s < 32; ++s) {
                const int i = blk * 32 + s;
                const int32_t xb = (int32_t)((bits >> s) & 1u);
                if (i < n) {
                    const int32_t v2 = 2 * d.hprof[i] + F[s];
                    pacc += (int64_t)(v2 & -xb);
                } else if (i < n_ext) {
                    sval += xb << (i - n);
                }
            }
#pragma unroll
            for (int w = 0; w < 4; ++w) swap_halves(x[0][w], x[0][w + 4]);
            rotate_chunks<NB>(x);
        }
        const int bt = b0;
        b0 = b1;
        b1 = bt;
        __syncthreads();
    }
    if (live) {
        d.rprofit[r] = pacc / 2;
        d.rfeas[r] = v.g <= sval ? 1 : 0;
        d.rg[r] = v.g;
        if constexpr (PT) d.rslot[r] = slot;
    }
}

}  // namespace pbit
