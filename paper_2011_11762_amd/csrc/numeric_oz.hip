// The Ozaki mode's leaf-product kernels, compiled apart from the other modes.
//
// Their integer MFMA accumulators (four int32 per 16 x 16 tile and pair
// group set) must be read by vector instructions at the end of every leaf,
// to be scaled and added to the FP64 accumulators.  This unit is built with
// the MFMA forms that keep accumulators in ordinary vector registers
// (-mllvm -amdgpu-mfma-vgpr-form, see build.py), which saves the copy of
// every accumulator out of the accumulation registers before each of those
// per-leaf additions.  The other modes' kernels keep their accumulators in
// the accumulation registers (numeric.hip).
#define QB_K5_OZAKI_UNIT 1
#include "numeric.hip"
