// Descriptor of one problem of the batched persistent solver (see batch.h): everything its
// workgroup reads, in device memory of the problem's workspace, filled by the host before
// each batched call; and the results the workgroup writes back.
#pragma once

#include "internal.h"

namespace gllmg {

constexpr int kBatchMaxLevels = 16;
constexpr int kBatchHist = 1024;       // residual history capacity (maxit < kBatchHist)
constexpr int kBatchThreads = 512;     // threads per workgroup (one problem)
constexpr int kBatchMaxProbs = 256;    // problems per launch (kernel argument size)
constexpr int kBatchLdsBytes = 96 * 1024;
// Problems up to this many fine-level nodes are solved by one workgroup each; larger ones take
// the stream path. Measured on 4^3-element batches (MI355X): one workgroup per problem is 12x
// faster than the streams at 729 nodes and 2.8x at 4913, but 2.5x slower at 35,937 (a single
// workgroup's element passes run one after the other with little latency hidden).
constexpr int64_t kBatchMaxNodes = 10000;

// Per level: everything the solve reads, in device memory of the problem's workspace.
struct BatchLevel {
  Grid g;
  int n, has_coarse, nch, pad;
  int64_t nint;
  double theta, delta;  // Chebyshev interval [cheb_lo lambda, lambda]: center and half-width
  const double* G64;
  const float* G32;
  const double* D64;
  const float* D32;
  const double* dinv64;
  const float* dinv32;
  const double* P64;  // transfer to the next coarser level
  const float* P32;
  const double* Ainv64;
  const float* Ainv32;
  void* vb[2];
  void* vx[2];
  void* vr[2];
  void* vd[2];
  void* vd2[2];
};

struct BatchProblem {
  // set up once
  int nlev, smoother, nu_pre, nu_post, vprec, pad0;
  double omega;
  void* F;
  const void* zero;
  double *pr, *pz, *pp, *ph, *pt;
  BatchLevel L[kBatchMaxLevels];
  // per call
  const double* b;
  double* x;
  double rtol;
  int maxit, mode;
  // results
  int iters, status;  // status 0 converged, 1 maximum iterations, 2 breakdown
  double n0, nr, relres_true;
  long long applies[kBatchMaxLevels];
  double hist[kBatchHist];
};

struct BatchArgs {
  BatchProblem* p[kBatchMaxProbs];
};

// host: launch the persistent solver of finest order n0 (2..17) for `count` problems
template <int N0>
void launch_batch_n(const BatchArgs& a, int count, hipStream_t s);
void launch_batch(int n0, const BatchArgs& a, int count, hipStream_t s);

}  // namespace gllmg
