#pragma once
#include "host.h"

namespace hs {

struct SoftmaxOpts {
    int variant = 0;          // 0 = SM (Algorithm SM), 1 = SM version B
    int k = 0;                // iterations; 0 = ceil(log M - log ln n)
    int exp_degree = 15;
    int inv_degree_first = 15;
    int inv_degree_mid = 15;
    int inv_degree_last = 31;
    int debug_stop = -1;      // >= 0: return y after that iteration (0 = after exp)
};

struct SoftmaxStats {
    int k = 0;
    int bootstraps = 0;       // ciphertext bootstraps (a batch of m counts m)
    int levels_left = 0;
};

int theorem_k(int n, double M);
// Softmax of the L = m N0 / n vectors packed in the batch x (Section 4.2
// layout); inputs in [-M, 0].  Returns the batch of outputs.
Ct softmax(Context& c, const Ct& x, int n, double M, const SoftmaxOpts& o, SoftmaxStats* stats);

bool can_bootstrap(const Context& c);
// Refresh x (any level) to the top user level; `bound` bounds |slot values|.
Ct bootstrap(Context& c, const Ct& x, double bound);
Ct bootstrap_stage(Context& c, const Ct& x, double bound, int stop);

}  // namespace hs
