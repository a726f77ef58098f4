// Quasi-1D kernel set (placeholder until the batched quasi-1D kernels land).
#include "ctx.h"

namespace tdslda {
std::unique_ptr<Engine> make_q1d_f64(int) { return nullptr; }
std::unique_ptr<Engine> make_q1d_f32(int) { return nullptr; }
}  // namespace tdslda
