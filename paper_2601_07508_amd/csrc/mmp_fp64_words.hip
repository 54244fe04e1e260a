// One (u, v) word pair of the fused FP64-word kernel, selected at build time
// by MMP_U and MMP_V, so that the pairs compile in parallel.
#include "fp64_words_kernel.h"

#if !defined(MMP_U) || !defined(MMP_V)
#error "build with -DMMP_U=<u> -DMMP_V=<v>"
#endif

#define MMP_CAT2(a, b, c) a##b##_##c
#define MMP_CAT(a, b, c) MMP_CAT2(a, b, c)

namespace mmp {

int MMP_CAT(launch_fp64_words_, MMP_U, MMP_V)(int tile_id, const Fp64Batch& a, void* stream) {
  using namespace fp64w;
  static_assert(MMP_U * MMP_V <= kMaxWordProducts, "unsupported word pair");
  constexpr int UV = MMP_U * MMP_V;
  hipStream_t s = (hipStream_t)stream;
  (void)UV;
  // k-steps per in-loop reduction: S / 4 for S in {4, 8}, else 4 (whole
  // stages); padded stages when a block leaves zero slots (L < S <= 16);
  // correction-free in-loop reductions or not; every product of a batch has
  // the same class (fp64_class)
  const int cls = fp64_class(a.job[0].S, a.job[0].L, a.job[0].lazy != 0);
  const int fe = cls >> 2;
  const bool pad = (cls & 2) != 0;
  const bool lazy = (cls & 1) != 0;
#define MMP_FE(ID_, FE_)                                                                       \
  if (fe == FE_) {                                                                             \
    if (pad) return lazy ? launch_shape<MMP_U, MMP_V, ID_, FE_, true, true>(a, s)              \
                         : launch_shape<MMP_U, MMP_V, ID_, FE_, true, false>(a, s);            \
    return lazy ? launch_shape<MMP_U, MMP_V, ID_, FE_, false, true>(a, s)                      \
                : launch_shape<MMP_U, MMP_V, ID_, FE_, false, false>(a, s);                    \
  }
#define MMP_SHAPE(ID_) \
  if (tile_id == ID_) { \
    MMP_FE(ID_, 1)      \
    MMP_FE(ID_, 2)      \
    MMP_FE(ID_, 4)      \
  }
  MMP_SHAPE(1)
  MMP_SHAPE(2)
  MMP_SHAPE(3)
#undef MMP_SHAPE
#undef MMP_FE
  return (int)hipErrorInvalidValue;
}

}  // namespace mmp
