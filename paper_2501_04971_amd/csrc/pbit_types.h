// Internal types shared by the host side of libpbit and its HIP kernels.
#pragma once
#include <stdint.h>

namespace pbit {

// Threshold table over beta*I in [-9, 9] at a 2^-8 step.
constexpr int kThetaHalf = 2304;
constexpr int kThetaLen = 2 * kThetaHalf + 1;
constexpr int kThetaBytes = 18448;          // kThetaLen * 4 rounded up to 16 bytes
constexpr int kXLen = 4609;                 // replica-exchange table: exp(j / 256), j = -4608 .. 0
constexpr int kMaxM = 32;                   // constraints per instance
constexpr int kMaxQuadBlocks = 11;          // quadratic kernel: n_ext <= 352
constexpr int kMaxWords = 64;               // linear kernel: n_ext <= 2048
constexpr int kWave = 64;
constexpr int kSnapshotBytes = 176;  // per-member record of batch snapshots
constexpr int kBatchSplit = 0x100;   // work-item code flag: split (1 + 3 waves, 64 replicas) linear tile
// producer/consumer kernels: double-buffered threshold ring (32 sites x 64 lanes)
constexpr size_t kRingBytes = 2 * 32 * 64 * 8;

// Per-sweep constants of the threshold on the field itself used by the split
// kernels (see field_threshold): for B_t > 0, A = floor(2^E / B_t) =
// a_hi 2^31 + a_lo, rho = 2^E mod B_t and rb = rho / B_t as a double, with
// E = S' - 1 (S' = S + u the shift of the carried field); sat = 1 when the
// threshold is +-2^62 by the sign alone (B_t = 0, or A >= 2^62); fast = 1 when
// A < 2^48 (then |n A| < 2^62 for every |n| < 2^14: field_threshold_fast).
struct ZtSweep {
    int32_t a_lo, a_hi, rho, bt;
    double rb;
    int32_t sat;
    int32_t fast;   // 1: A < 2^48, so n a_hi fits 31 bits and nothing saturates
};

// Everything a kernel needs about one instance; passed by value.
struct DevInstance {
    // constants written once at create
    const int8_t *J;          // quadratic: slabs of 32 rows x (n_pad + 16) bytes, slab stride 1 KB x (nb + 1)
    const int32_t *theta;     // [kThetaLen]
    const int32_t *Btab;      // [T] beta grid
    const ZtSweep *zsweep;    // [T] constants of the field thresholds (split kernels)
    const int32_t *bladder;   // [64] parallel tempering ladder on the beta grid
    const int32_t *xtab;      // [4609] exchange acceptance 2^24 exp(j / 256), j = -4608 .. 0
    const int32_t *acol;      // [n_ext][m] extended constraint coefficients, site-major
    const int64_t *kbase;     // [n_ext] 256 s_g^2 h_i - Sa_i
    const int64_t *sa2;       // [n_ext] 2 Sa_i,  Sa_i = s_f Pq |a_i|^2
    const int64_t *b;         // [m]
    const int32_t *hprof;     // [n] item profits
    const int32_t *slack_off; // [m] first slack site of constraint k
    const int32_t *slack_q;   // [m] slack bits of constraint k
    // state
    int64_t *site;            // [n_pad][4] per-site record: K0, K1, c, meta (see below)
    int64_t *lam_acc;         // [m] lambda_n on a 2^-32 grid
    int32_t *lam_q;           // [m] lambda_n on a 2^-8 grid
    int32_t *round_k;         // [1] rounds completed
    int64_t *G;               // [m] sum of residuals of the last round
    int64_t *best;            // [4] profit, round, replica, valid
    uint32_t *best_x;         // [words]
    int32_t *feas_count;      // [1] feasible replicas of the last round
    uint32_t *lam_sat;        // [1] bit k set once lambda_k has been held at +-lq_max (sticky)
    int32_t *rounds_left;     // [1] multiplier steps still to run (batch members), or null
    // per-replica outputs of the last round
    uint32_t *rx;             // [R][words]
    int32_t *rg;              // [R][m]
    int64_t *rprofit;         // [R]
    int32_t *rfeas;           // [R]
    int32_t *rslot;           // [R] final ladder position (parallel tempering; 0 otherwise)
    // scalars
    int32_t n, m, n_ext, n_pad, words, owords, R, T, S, nq;
    int32_t sg2;              // 2^u s_g^2 (quadratic kernel; < 2^31)
    int32_t k2;               // 2^u 2 s_f Pq (< 2^31)
    int32_t zsh;              // u: fields are carried as 2^u Z so that S + u >= 34
    int32_t ish;              // S + u - 32 (>= 2)
    int64_t irnd;             // 2^(S + u - 33): rounding term of the index, in units of 2^32
    int32_t hclo, hchi;       // clamp of the index's high word before the final shift
    int64_t sfsg;             // s_f s_g
    int64_t lq_max;
    int64_t eta_num;
    int64_t lam_den;          // eta_den * R * s_g
    uint32_t seed_lo, seed_hi, inst_id;
    int32_t eta_h;            // diminishing step eta H / (H + k); 0: constant eta
    int32_t eta_kcap;         // largest k used in H + k (keeps lam_den (H + k) < 2^62)
    int32_t pt;               // parallel tempering chain length L (0: annealing)
};

// Per-site record (4 x int64), i < n_pad:
//   K0, K1  2^u (256 s_g^2 h_i - s_f s_g a_i.lq - Sa_i (1 - 2 x_i)) for x_i = 0, 1
//   c       2^u (256 s_g^2 W_{i,i-1} - 2 s_f Pq a_i.a_{i-1}): change of Z_i when
//           site i-1 flips from 0 to 1 (0 where i-1 is not the preceding visit)
//   meta    low word a_i (one-constraint kernel), high word -1 for a real
//           site and 0 for padding
enum Variant { kQuad = 0, kLinear = 1, kLinearWide = 2 };

}  // namespace pbit
