// Segment-wise restarted flexible GMRES shared by gmres_solve (the columns
// of one system) and gmres_solve_batch (the problems of a batch).
#pragma once
#include <functional>
#include <vector>

#include "handle.h"

namespace hlu {

struct GmresSystem {
  int32_t nseg = 0;                  // independent systems
  std::vector<int64_t> off, len;     // segment c: elements [off[c], off[c] + len[c]) of a block
  int64_t total = 0;                 // elements of one vector block
  // whole-block operator and preconditioner: out = A in, out = M^{-1} in
  std::function<void(const double*, double*)> matvec, precond;
  // error word of the preconditioner's persistent launches (ctr[3]), read
  // at every synchronisation of the iteration; may be null
  int32_t* d_err = nullptr;
};

// Device bytes gmres_core needs for blocks of `total` elements.
size_t gmres_core_bytes(int64_t total, int32_t nseg, int32_t restart);

// b: right-hand sides (one block); x: result block (overwritten); info: one
// record per segment.  Synchronises the stream.
void gmres_core(const GmresSystem& sys, const double* b, double* x, const hlu_gmres_opts* o, void* d_work,
                hlu_gmres_info* info, hipStream_t s);

void check_gmres_opts(const hlu_gmres_opts* o);

}  // namespace hlu
