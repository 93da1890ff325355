// su2_learned.hpp -- internal interface of the learned block proposal
// (network, loss gradient, Adam, block move) to the C-ABI facade.
#pragma once

#include "su2_launch.hpp"

namespace su2 {
namespace lp {

// Network workspace: input features, three activations, outputs and their
// gradients, two gradient buffers, partial sums.
struct WorkLayout {
    uint64_t feat, a1, a2, a3, y, dy, dz_a, dz_b, part, loss_part, total;
};

int param_count();
WorkLayout work_layout(const int32_t n[4]);
void launch_forward(const LaunchArgs &a, const float *params, char *work, float *y, hipStream_t st);
void launch_loss_grad(const LaunchArgs &a, double beta, const float *params, char *work, float *grad, double *loss,
                      hipStream_t st);
void launch_adam(float *p, const float *grad, float *m, float *v, uint32_t n, int step, float lr, float b1, float b2,
                 float eps, hipStream_t st);
void launch_block_move(const LaunchArgs &a, double beta, uint64_t seed, uint32_t step, int parity, int colour,
                       const float *y, uint32_t *accepted, hipStream_t st);

} // namespace lp
} // namespace su2
