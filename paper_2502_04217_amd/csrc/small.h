// Batches of small problems, one workgroup per problem (small.hip).
#pragma once

#include "csipm_internal.h"

namespace csipm {

// the largest extent of a small problem (direct DFTs: L^2 work per pencil)
constexpr int kSmallMaxExtent = 64;
// the spectrum buffers (one, or two when an extent takes the direct DFT) of
// a grid sit in LDS when they take at most this many bytes
constexpr long long kSmallLdsBytes = 131072;

// the options the small solver reads (those of csipm_options it uses)
struct SmallOpts {
  double tol;
  int max_iter;
  int cg_max;
  double cg_rtol;
  double cg_atol;
  double sigma;
  double tau;
};

bool small_supported(int n1, int n2, int n3);
// workspace bytes of one problem (a multiple of 256)
size_t small_problem_bytes(int n1, int n2, int n3);
// one launch of count workgroups; tw holds the tables exp(-2 pi i q / L) of
// L = n1, n2, n3 in that order
hipError_t small_launch(int n1, int n2, int n3, int count, const double* signals, const uint8_t* observed,
                        const double* lambdas, double lambda_frac, double* beta_out, double* info, char* ws,
                        const cx<double>* tw, const SmallOpts& o, hipStream_t s);

}  // namespace csipm
