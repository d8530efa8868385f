// Staged-precision instantiations of the persistent batch kernel (fp16,
// two-word bf16, two-word fp16), compiled apart from the float32 ones so
// that the two halves build in parallel.
#include "fobf_batch_kern.h"

namespace fobf {

namespace {
template <int PREC>
BatchLauncher staged_for(int cidx) {
  switch (cidx) {
    case 0: return launch_batch<PREC, 2, 4>;
    case 1: return launch_batch<PREC, 5, 5>;
    default: return launch_batch<PREC, 6, 7>;
  }
}
}  // namespace

BatchLauncher batch_launcher_staged(int prec, int cidx) {
  switch (prec) {
    case FOBF_FP16_STAGE: return staged_for<FOBF_FP16_STAGE>(cidx);
    case FOBF_BF16_STAGE: return staged_for<FOBF_BF16_STAGE>(cidx);
    default: return staged_for<FOBF_FP16X2_STAGE>(cidx);
  }
}

}  // namespace fobf
