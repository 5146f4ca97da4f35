// Solver entry used by the C ABI (capi.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/slamg.h"
#include "common.h"

namespace slamg {

struct SolverError {
  int code;
  std::string msg;
};

// Prepared problem (after transposition / empty-row removal): host CSR with int32 indices and,
// optionally, device-resident copies owned by a prepared-matrix handle.
struct Problem {
  int kind = SLAMG_SVD, target = SLAMG_DOMINANT, nb = 1;
  HCsr A;
  const DCsr* dA = nullptr;    // device A (values + pattern), or null: uploaded by the solve
  const DCsr* dAt = nullptr;   // device A^t (SVD)
  const DCsr* dB = nullptr;    // finest B = I as CSR (SVD: m x m; eigen: values on A's pattern)
  const DCsr* dC = nullptr;    // finest C = I (SVD)
  // device outputs (column-major, original row numbering); null U: outputs go to the host
  double* outU = nullptr;
  double* outV = nullptr;
  long ldU = 0, ldV = 0;
  const int* keepU = nullptr;  // prepared row -> original row of outU
  const int* keepV = nullptr;
  bool swapUV = false;         // prepared U is the caller's V (m < n handled through A^t)
};

struct SolveOutput {
  std::vector<double> sigma;   // nb
  std::vector<double> U, V;    // row-major m x nb, n x nb (prepared sizes)
  slamg_report rep;
  int status = ST_OK;
};

// Runs the whole method on the device; throws SolverError on failure.
void run_solver(hipStream_t stream, size_t budget, const Problem& pb, const slamg_params& p,
                const double* init_tests, SolveOutput& out);

uint64_t splitmix64_next(uint64_t& state);
double splitmix64_uniform(uint64_t seed, uint64_t k);   // k-th output (k >= 1) mapped to [-1, 1)

}  // namespace slamg
