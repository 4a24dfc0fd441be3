// Host-side view of the layer-pipelined incremental kernels (gna_pipe.hip): their
// instantiations per precision, feature width and workgroup size.
#pragma once

namespace gna {

struct PipeKern {
  const void* eloc = nullptr;    // k_eloc_pipe
  const void* sweep = nullptr;   // k_sweep_pipe
  int maxt = 0;                  // tile registers per wave
  int ncopy = 0;                 // ring-row vectors per thread held across a barrier
};

// prec: a gna_precision value; nt: 512 or 1024 threads.  Null kernels when that
// combination has no pipelined instantiation.
PipeKern pipe_pick(int prec, int F, int nt);

}  // namespace gna
