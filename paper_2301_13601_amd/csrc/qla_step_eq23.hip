// Instances of the fused step kernel for the Eq. (23) placement of the
// potentials.
#include "qla_step.hpp"

namespace qla_dev {

StepImpl pick_step_eq23(bool vec, bool wide, bool pot) {
  constexpr int C = 2;
  constexpr int M = 0;
  if (vec) {
    if (wide) return pot ? impl<C, true, true, M, true>() : impl<C, true, true, M, false>();
    return pot ? impl<C, true, false, M, true>() : impl<C, true, false, M, false>();
  }
  if (wide) return pot ? impl<C, false, true, M, true>() : impl<C, false, true, M, false>();
  return pot ? impl<C, false, false, M, true>() : impl<C, false, false, M, false>();
}

}  // namespace qla_dev
