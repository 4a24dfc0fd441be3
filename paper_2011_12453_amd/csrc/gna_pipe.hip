// Instantiations of the layer-pipelined incremental kernels (gna_pipe.h), compiled
// apart from gna.hip so that the two translation units build in parallel.
#include <hip/hip_runtime.h>

#include "gna.h"
#include "gna_pipe.h"
#include "gna_pipe_api.h"

namespace gna {

namespace {

template <class P, int F, int MAXT, int NT, int NCOPY>
PipeKern pipe_make() {
  PipeKern k;
  k.eloc = reinterpret_cast<const void*>(&k_eloc_pipe<P, F, MAXT, NT, NCOPY>);
  k.sweep = reinterpret_cast<const void*>(&k_sweep_pipe<P, F, MAXT, NT, NCOPY>);
  k.maxt = MAXT;
  k.ncopy = NCOPY;
  return k;
}

// 8 waves (7 computing) of up to six tiles, or 16 waves (15 computing) of up to two
template <class P, int F>
PipeKern pipe_nt(int nt) {
  if (nt == 1024) return pipe_make<P, F, 2, 1024, 2>();
  return pipe_make<P, F, 6, 512, 4>();
}

}  // namespace

PipeKern pipe_pick(int prec, int F, int nt) {
  switch (prec) {
    case GNA_FP32:
      if (F == 16) return pipe_nt<PF32, 16>(nt);
      if (F == 32) return pipe_nt<PF32, 32>(nt);
      return pipe_nt<PF32, 64>(nt);
    case GNA_BF16_1X:
      if (F == 16) return pipe_nt<PBF161, 16>(nt);
      if (F == 32) return pipe_nt<PBF16W1, 32>(nt);
      return pipe_nt<PBF16W1, 64>(nt);
    case GNA_BF16:
      if (F == 16) return pipe_nt<PBF16, 16>(nt);
      if (F == 32) return pipe_nt<PBF16W, 32>(nt);
      return pipe_nt<PBF16W, 64>(nt);
    default:
      return PipeKern{};
  }
}

}  // namespace gna
