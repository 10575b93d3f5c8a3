// Annealing run for instances with pair profits (quadratic knapsack, one
// constraint): the p-bit machine of Sec. III-B, one replica per lane.
//
// Field of site i for replica r (Eq. Ii_eq in the 0/1 form, all integers):
//   Z_i = 256 s_g^2 F_i + K_{x_i,i} - 2 s_f Pq a_i g
// with F_i = sum_j W_ij x_j, g = a.x - b the residual, and K_{0,i}, K_{1,i} the
// per-site constants of the current lambda (h_i, the penalty's self term and
// the Lagrange term folded in).  The update of Eq. mi_eq is
//   x_i <- [u24 < Theta[round(beta_t Z_i / (2 s_f s_g^2))]].
//
// Layout: the threshold table and the per-site records sit in LDS; the int8
// profit block W (n_pad x n_pad, rows padded by 16 bytes) stays in global
// memory (L2-resident) and is streamed through LDS one 32-row slab per block,
// double-buffered: the next slab's pieces are loaded and stored to the free
// buffer between the visits of the current block.  Each lane keeps its replica's state as
// n_pad bytes in VGPRs.  Sites are visited in blocks of 32: at the start of a
// block the 32 fields of the block are computed for all 64 replicas of the
// wave with int8 MFMA, over every column except the block's own earlier sites
// (W[i, j] with j in the block and j < i is left out: the host stores that
// strictly lower part of the diagonal chunk apart, see diag_arow); the visit of
// site i adds it with packed int8 dot products against the current state bytes
// of the block (W[i, blk] . x), so that a decision feeds the next visit through
// one state-byte update and one dot product.  The penalty is never expanded
// into couplings: the constraint enters through the residual g.
//
// Register layout of the state: chunk c (sites 32c..32c+31) is 8 dwords per
// lane.  Outside its own block a chunk is stored in the MFMA B-operand layout
// (lanes 0..31 hold sites 0..15 of replicas 0..31 / 32..63, lanes 32..63 sites
// 16..31), which one permlane32 swap per dword pair converts to and from the
// owner layout (lane r holds all 32 bytes of replica r).  The chunk of the
// current block is kept at register position 0: positions rotate by one chunk
// per block, so all indexing is static.
#pragma once
#include <utility>

#include "device_common.h"

namespace pbit {

// Accumulators of the two 32-replica halves (row 8(v/4) + 4(lane/32) + v%4,
// column lane%32) -> owner layout (lane r holds the 32 fields of replica r).
__device__ __forceinline__ void fields_from_acc(const v16i &acc0, const v16i &acc1, int32_t (&F)[32])
{
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        uint32_t lo = (uint32_t)acc0[v], hi = (uint32_t)acc1[v];
        swap_halves(lo, hi);
        F[8 * (v >> 2) + (v & 3)] = (int32_t)lo;
        F[8 * (v >> 2) + 4 + (v & 3)] = (int32_t)hi;
    }
}

// MFMA A operand of a slab's diagonal chunk without its strictly lower part
// (W[i, j], j >= i, both in the slab's block): the host stores columns 0..15 of
// row r in the row's 16 padding bytes and columns 16..31 at 32 LS + 16 r, so
// lane l (row l % 32, columns 16 (l / 32) ..) reads 16 bytes from there.
template <int NB>
__device__ __forceinline__ const int8_t *diag_arow(const int8_t *slab, int lane)
{
    constexpr int LS = NB * 32 + 16;
    const int row = lane & 31;
    return slab + (lane < 32 ? row * LS + NB * 32 : 32 * LS + row * 16);
}

// Block fields F[blk*32 + s] = sum_j W[blk*32+s, j] x_j for the 64 replicas of
// the wave, except (FULL = false) the terms j = blk*32 + s' with s' < s (slab
// holds rows blk*32..blk*32+31 of W).
template <int NB, bool FULL = false>
__device__ __forceinline__ void block_fields(const int8_t *slab, int blk, const uint32_t (&x)[NB][8],
                                             int32_t (&F)[32])
{
    constexpr int LS = NB * 32 + 16;
    const int lane = threadIdx.x & 63;
    const int8_t *arow = slab + (lane & 31) * LS + (lane >> 5) * 16;
    v16i acc0 = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    v16i acc1 = acc0;
#pragma unroll
    for (int p = 0; p < NB; ++p) {
        int c = p + blk;
        c = c >= NB ? c - NB : c;
        // p = 0 is the block's own chunk
        const v4i A = *reinterpret_cast<const v4i *>(p == 0 ? diag_arow<NB>(slab, lane) : arow + c * 32);
        const v4i B0 = {(int)x[p][0], (int)x[p][1], (int)x[p][2], (int)x[p][3]};
        const v4i B1 = {(int)x[p][4], (int)x[p][5], (int)x[p][6], (int)x[p][7]};
        acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B1, acc1, 0, 0, 0);
        if (FULL && p == 0) {
            // the strictly lower part, kept in the chunk's own place
            const v4i L = *reinterpret_cast<const v4i *>(arow + c * 32);
            acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(L, B0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(L, B1, acc1, 0, 0, 0);
        }
    }
    fields_from_acc(acc0, acc1, F);
}

template <int NB>
__device__ __forceinline__ void rotate_chunks(uint32_t (&x)[NB][8])
{
    uint32_t tmp[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) tmp[w] = x[0][w];
#pragma unroll
    for (int p = 0; p + 1 < NB; ++p)
#pragma unroll
        for (int w = 0; w < 8; ++w) x[p][w] = x[p + 1][w];
#pragma unroll
    for (int w = 0; w < 8; ++w) x[NB - 1][w] = tmp[w];
}

// Slab b of W = rows 32b..32b+31, LS bytes each, stored with a stride of
// 1 KB x (NB + 1) (the tail of each slab is padding).  Whole-workgroup copy
// into an LDS buffer, used outside the visit loop.
template <int NB>
__device__ __forceinline__ void copy_slab(const int8_t *J, int b, int8_t *dst)
{
    constexpr int SLABP = 1024 * (NB + 1);
    const uint4 *src = reinterpret_cast<const uint4 *>(J + (size_t)b * SLABP);
    uint4 *d = reinterpret_cast<uint4 *>(dst);
    for (int e = threadIdx.x; e < SLABP / 16; e += blockDim.x) d[e] = src[e];
}

template <int NB>
constexpr size_t quad_lds_bytes()
{
    return (size_t)kThetaBytes + (size_t)NB * 32 * 32 + 2 * (size_t)1024 * (NB + 1);
}

// Registers of one block of 32 visits, shared by the unrolled steps.
struct BlockVisit {
    const int64_t *rec;      // per-site records of the block
    const int8_t *wblk;      // LDS: W[blk*32 .., blk*32 ..]
    const int32_t *th;       // LDS threshold table
    int32_t F[32];           // block fields at the block start (without the lower in-block terms)
    uint32_t rnd[4];
    int32_t g;
    int32_t Bt, ish, hclo, hchi;
    int64_t E;               // parallel tempering: D (L(x) - L(0)) carried as 2^u
    int64_t irnd, sg2, k2;
    uint32_t cbase, kround, inst, seed_lo, seed_hi;
    uint64_t m2;
    int blk;
    // streaming of the next block's slab of W: 1 KB pieces, piece c handled by
    // wave c % nw; lane l moves bytes 16 l .. 16 l + 15 of each piece
    const int8_t *jnext;     // global: next slab
    int8_t *lnext;           // LDS: buffer that receives it
    int wave, nw;
    uint4 pf[5];             // pieces in flight
};

// Piece j of this wave (c = wave + j WPB, clamped to the last piece so the
// schedule has no branches; a clamped piece is a repeated identical store) is
// loaded at visit 2j and stored at visit 2j + 8.  The store comes first so that
// its wait covers only the loads issued eight visits earlier.
template <int s, int NB, int WPB>
__device__ __forceinline__ void stream_slab(BlockVisit &v)
{
    constexpr int PIECES = NB + 1;  // slab stride in global memory and LDS: 1 KB x (NB + 1)
    constexpr int JW = (PIECES + WPB - 1) / WPB;
    const int lane = threadIdx.x & 63;
    if constexpr ((s & 1) == 0 && s >= 8 && (s - 8) / 2 < JW) {
        constexpr int j = (s - 8) / 2;
        const int c = min(v.wave + j * WPB, PIECES - 1);
        *reinterpret_cast<uint4 *>(v.lnext + c * 1024 + lane * 16) = v.pf[j % 5];
    }
    if constexpr ((s & 1) == 0 && s / 2 < JW) {
        constexpr int j = s / 2;
        const int c = min(v.wave + j * WPB, PIECES - 1);
        v.pf[j % 5] = *reinterpret_cast<const uint4 *>(v.jnext + c * 1024 + lane * 16);
    }
}

// One visit of site s: its threshold index is computed from the current state
// right before the decision.  The field adds W[s, s'] x_s' for the block's
// earlier sites s' < s to the block-start field (the row's entries at s' >= s
// are zero there, so whole state words can be used).  With parallel tempering
// the replica's energy follows every flip: Z is -D times the energy change of
// switching the site on, so a flip by delta changes D L by -delta Z.
template <int s, int LS, int WPB, bool PT = false>
__device__ __forceinline__ void visit_site_direct(BlockVisit &v, uint32_t (&xc)[8], const uint32_t (&x0)[8])
{
    stream_slab<s, (LS - 16) / 32, WPB>(v);
    // old states come from the block-start copy (site s changes only at its own
    // visit), which keeps the record loads off the chain of decisions
    const uint32_t xo = (x0[s >> 2] >> (8 * (s & 3))) & 1u;
    const int64_t *cur = v.rec + 4 * s;
    int32_t f = v.F[s];
    const uint32_t *wrow = reinterpret_cast<const uint32_t *>(v.wblk + s * LS);
#pragma unroll
    for (int w = 0; w < (s + 3) / 4; ++w) f = __builtin_amdgcn_sdot4((int)wrow[w], (int)xc[w], f, false);
    const int64_t meta = cur[3];
    const int64_t Z = cur[xo] + (int64_t)(f * 256) * v.sg2 - (int64_t)__mul24((int32_t)meta, v.g) * v.k2;
    const uint32_t thr = (uint32_t)v.th[theta_index(Z, v.Bt, v.ish, v.irnd, v.hclo, v.hchi) + kThetaHalf] &
                         (uint32_t)(meta >> 32);
    if constexpr ((s & 3) == 0)
        philox_block(v.cbase + (uint32_t)((v.blk * 32 + s) >> 2), v.kround, v.m2, v.inst, v.seed_lo,
                     v.seed_hi, v.rnd);
    const uint32_t u24 = v.rnd[s & 3] >> 8;
    const uint32_t xn = u24 < thr ? 1u : 0u;
    const int32_t delta = (int32_t)xn - (int32_t)xo;
    xc[s >> 2] += (uint32_t)delta << (8 * (s & 3));
    v.g += __mul24(delta, (int32_t)meta);
    if constexpr (PT) v.E = delta > 0 ? v.E - Z : (delta < 0 ? v.E + Z : v.E);
}

#ifndef PBIT_SCHED_WINDOW
#define PBIT_SCHED_WINDOW 4
#endif

// Scheduling fence every PBIT_SCHED_WINDOW visits: keeps the compiler from
// hoisting the loads of all 32 unrolled visits (which would cost registers and
// therefore waves per SIMD) while leaving room to overlap neighbouring visits.
template <int s, int WIN = PBIT_SCHED_WINDOW>
__device__ __forceinline__ void visit_fence()
{
    if constexpr ((s + 1) % WIN == 0) __builtin_amdgcn_sched_barrier(0);
}

template <int LS, int WPB, bool PT, int... S>
__device__ __forceinline__ void visit_block(BlockVisit &v, uint32_t (&xc)[8], std::integer_sequence<int, S...>)
{
    const uint32_t x0[8] = {xc[0], xc[1], xc[2], xc[3], xc[4], xc[5], xc[6], xc[7]};
    ((visit_site_direct<S, LS, WPB, PT>(v, xc, x0), visit_fence<S>()), ...);
}

// Replica exchange after sweep t (parallel tempering, chains of L lanes inside
// a wave, L a power of two dividing 64).  Lane l of a chain is the keeper of
// ladder position tau = l mod L: it knows `owner`, the lane whose replica is at
// tau.  For the pairs (tau, tau + 1) with tau = t mod 2 the keeper of tau draws
// from Philox(t, k | 2^31, r, instance), r its own replica index (= c L + tau),
// and decides: swap when j = floor(2 (B_tau - B_tau+1)(E_a - E_b) / 2^S') >= 0
// or u24 < X[j] (j >= -4608, X[j] = 2^24 exp(j / 256)), E the carried energies
// of the replicas a at tau and b at tau + 1, S' = ish + 32.  The keepers then
// take their new owners and every replica learns its new position.
__device__ __forceinline__ void pt_exchange(const DevInstance &d, int t, uint32_t kround, uint64_t m2, int64_t E,
                                            int32_t &owner, int32_t &slot)
{
    const int L = d.pt;
    const int lane = threadIdx.x & 63;
    const int tau = lane & (L - 1);
    const int up = tau + 1 < L ? lane + 1 : lane;  // keeper of tau + 1
    const int32_t own_lo = owner;
    const int32_t own_hi = __shfl(owner, up, 64);
    const int32_t elo_l = __shfl((int32_t)(uint32_t)E, own_lo, 64), elo_h = __shfl((int32_t)(E >> 32), own_lo, 64);
    const int32_t ehi_l = __shfl((int32_t)(uint32_t)E, own_hi, 64), ehi_h = __shfl((int32_t)(E >> 32), own_hi, 64);
    const int64_t ea = (int64_t)(((uint64_t)(uint32_t)elo_h << 32) | (uint32_t)elo_l);
    const int64_t eb = (int64_t)(((uint64_t)(uint32_t)ehi_h << 32) | (uint32_t)ehi_l);
    const bool pair = (tau & 1) == (t & 1) && tau + 1 < L;
    bool accept = false;
    if (pair) {
        // (B_tau - B_tau+1)(E_a - E_b) = (B_tau+1 - B_tau)(E_b - E_a), the first
        // factor in [0, 2^31) and |E_b - E_a| < 2^62
        const int32_t dB = d.bladder[tau + 1] - d.bladder[tau];
        const int64_t hq = field_hi(eb - ea, dB, 0);  // floor(dB dE / 2^32)
        const int64_t j = hq >> (d.ish - 1);            // floor(2 dB dE / 2^S')
        if (j >= 0) {
            accept = true;
        } else {
            uint32_t w[4];
            philox_block((uint32_t)t, kround | 0x80000000u, m2, d.inst_id, d.seed_lo, d.seed_hi, w);
            const int idx = j < -(kXLen - 1) ? 0 : (int)j + kXLen - 1;
            accept = (w[0] >> 8) < (uint32_t)d.xtab[idx];
        }
    }
    // the keeper of tau + 1 takes the lower replica when the pair below swapped
    const int down = tau > 0 ? lane - 1 : lane;
    const int acc_below = __shfl(accept ? 1 : 0, down, 64) & (tau > 0 ? 1 : 0);
    const int32_t own_below = __shfl(own_lo, down, 64);
    owner = accept ? own_hi : (acc_below ? own_below : own_lo);
    // every replica's position: the keeper of tau pushes tau to its owner's lane
    slot = __builtin_amdgcn_ds_permute(owner << 2, tau);
}

// One annealing run (T sweeps) of the replicas rbase + [0, 64 WPB) of instance
// d, followed by the scoring of the final states.  The workgroup has WPB
// waves; smem must hold quad_lds_bytes<NB>() bytes.
template <int NB, int WPB, bool PT = false>
__device__ __forceinline__ void quad_run(const DevInstance &d, int rbase, unsigned char *smem)
{
    constexpr int NP = NB * 32;        // padded spin count
    constexpr int LS = NP + 16;        // row stride of W (bytes)
    constexpr int SLAB = 1024 * (NB + 1);  // slab stride (rows of LS bytes plus padding)
    int32_t *th = reinterpret_cast<int32_t *>(smem);
    int64_t *site = reinterpret_cast<int64_t *>(smem + kThetaBytes);
    int8_t *slabs = reinterpret_cast<int8_t *>(smem + kThetaBytes + NP * 32);

    copy_slab<NB>(d.J, 0, slabs);
    for (int e = threadIdx.x; e < kThetaLen; e += blockDim.x) th[e] = d.theta[e];
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(d.site);
        uint4 *dst = reinterpret_cast<uint4 *>(site);
        for (int e = threadIdx.x; e < NP * 2; e += blockDim.x) dst[e] = src[e];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int r = rbase + threadIdx.x;
    const uint32_t kround = (uint32_t)d.round_k[0];
    const uint64_t m2 = (uint64_t)0xCD9E8D57u * (uint32_t)r;
    const int32_t *__restrict__ Btab = d.Btab;

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
    v.k2 = d.k2;
    v.kround = kround;
    v.inst = d.inst_id;
    v.seed_lo = d.seed_lo;
    v.seed_hi = d.seed_hi;
    v.m2 = m2;
    v.wave = threadIdx.x >> 6;
    v.nw = WPB;
#pragma unroll
    for (int w = 0; w < 4; ++w) v.rnd[w] = 0u;
    // parallel tempering: the replica's ladder position, the lane this lane
    // keeps track of (the one at ladder position lane mod L), its energy
    int32_t slot = 0, owner = lane;
    v.E = 0;
    if constexpr (PT) slot = lane & (d.pt - 1);

    // the two LDS slab buffers alternate every block; the block sequence wraps
    // from NB - 1 to 0 at each sweep, so the buffer index is a running toggle
    int buf = 0;
    for (int t = 0; t < d.T; ++t) {
        v.Bt = PT ? d.bladder[slot] : Btab[t];
        v.cbase = (uint32_t)t * (uint32_t)d.nq;
        for (int blk = 0; blk < NB; ++blk) {
            const int8_t *slab = slabs + buf * SLAB;
            // the next block's slab (block 0 again after the last one) streams in meanwhile
            v.jnext = d.J + (size_t)(blk + 1 < NB ? blk + 1 : 0) * SLAB;
            v.lnext = slabs + (buf ^ 1) * SLAB;
            block_fields<NB>(slab, blk, x, v.F);
#pragma unroll
            for (int w = 0; w < 4; ++w) swap_halves(x[0][w], x[0][w + 4]);

            v.rec = site + 4 * (blk * 32);
            v.wblk = slab + blk * 32;
            v.blk = blk;
            visit_block<LS, WPB, PT>(v, x[0], std::make_integer_sequence<int, 32>{});
#pragma unroll
            for (int w = 0; w < 4; ++w) swap_halves(x[0][w], x[0][w + 4]);
            rotate_chunks<NB>(x);
            buf ^= 1;
            __syncthreads();
        }
        if constexpr (PT) pt_exchange(d, t, kround, m2, v.E, owner, slot);
    }

    // Score the final state: profit = (sum_{i<n} x_i (2 h_i + F_i)) / 2 with
    // F = W x, slack value s = sum_q 2^q x_{n+q}; feasible iff g <= s.
    const int n = d.n, n_ext = d.n_ext;
    const bool live = r < d.R;
    int64_t pacc = 0;
    int32_t sval = 0;
    for (int blk = 0; blk < NB; ++blk) {
        const int8_t *slab = slabs + buf * SLAB;
        if (blk + 1 < NB) copy_slab<NB>(d.J, blk + 1, slabs + (buf ^ 1) * SLAB);
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
        buf ^= 1;
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
