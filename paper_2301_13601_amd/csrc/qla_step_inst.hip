// Instances of the fused step kernel for one placement of the potentials
// (QLA_MODE: 0 = Eq. (23), 1 = Eq. (28)) and one field triple (QLA_FIELDS:
// 0 = all six components, 1 = TM, 2 = TE). The build compiles this unit once
// per pair, in parallel.
#include "qla_step.hpp"

#if !defined(QLA_MODE) || !defined(QLA_FIELDS)
#error "QLA_MODE and QLA_FIELDS must be defined"
#endif

#define QLA_CAT2(a, b) a##b
#define QLA_CAT(a, b) QLA_CAT2(a, b)
#define QLA_PICK QLA_CAT(QLA_CAT(QLA_CAT(pick_step_m, QLA_MODE), _f), QLA_FIELDS)

namespace qla_dev {

StepImpl QLA_PICK(const StepChoice& ch) { return pick_step<QLA_MODE, QLA_FIELDS>(ch); }

}  // namespace qla_dev
