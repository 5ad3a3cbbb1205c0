#pragma once
#include "host.h"

namespace hs {

struct SoftmaxOpts {
    int variant = 0;          // 0 = SM (Algorithm SM), 1 = SM version B
    int k = 0;                // iterations; 0 = ceil(log M - log ln n)
    int exp_degree = 15;
    // 0 = by dimension (degrees 2^d - 1): n <= 256 the depths of the paper's
    // table of the auxiliary thread's level usage at n = 256 (Section 5: 6,
    // 5, 7); n <= 1024: 6, 6, 8; larger: 7, 7, 8
    int inv_degree_first = 0;
    int inv_degree_mid = 0;
    int inv_degree_last = 0;
    int debug_stop = -1;      // >= 0: return y after that iteration (0 = after exp)
    int power = 2;            // t of normalize-and-t-th-power (2, 3, 4; version B: 2)
    int newton_steps = 0;     // > 0: inverse roots by that many Newton steps from the polynomial
    int mask_mode = 0;        // 0: indicator of slots [0, L); 1: averaging (m / n on every slot)
    int approx = 0;           // normalisation polynomials: 0 weighted minimax, 1 Chebyshev interpolants
    int merge = 0;            // jobs > 1, version B: one auxiliary ciphertext for every job
};

struct SoftmaxStats {
    int k = 0;
    int bootstraps = 0;       // ciphertext bootstraps (a batch of m counts m)
    int levels_left = 0;
};

int theorem_k(int n, double M);
// Softmax of the L = m N0 / n vectors packed in the batch x (Section 4.2
// layout); inputs in [-M, 0].  Returns the batch of outputs.
// jobs > 1: x holds `jobs` independent batches of x.m / jobs ciphertexts each
// (same n, M), run in lockstep: the main-thread operations cover every
// ciphertext in each launch and the jobs' auxiliary ciphertexts form one batch
// (one key read per operation, one batched bootstrap).  Every operation acts
// per ciphertext, so each job's result equals its result alone.
Ct softmax(Context& c, const Ct& x, int n, double M, const SoftmaxOpts& o, SoftmaxStats* stats, int jobs = 1);

bool can_bootstrap(const Context& c);
// Refresh x (any level) to the top user level; `bound` bounds |slot values|.
// With mask_L > 0 the result is also multiplied by the 0/1 mask of slots
// [0, L) (folded into the last SlotToCoeff matrix, no extra level).
Ct bootstrap(Context& c, const Ct& x, double bound, int mask_L = 0);
Ct bootstrap_stage(Context& c, const Ct& x, double bound, int stop, int mask_L = 0);

}  // namespace hs
