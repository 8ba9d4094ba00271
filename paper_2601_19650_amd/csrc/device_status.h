// Device side of a call's status word, shared by the eigensolve and Cholesky kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace cbc {

// store `code` into the status word if it still holds CBC_OK (the first failure is kept)
__device__ inline void raise_status(int* status, int code) {
  if (status) atomicCAS(status, 0, code);
}

}  // namespace cbc
