// Device-resident batch of two-sided BiCG columns (internal to libmorx).
//
// A batch has `cap` column slots on one system.  Each slot holds one primal +
// dual (or shadow) recurrence, its own shift, right-hand sides, output
// pointers and its own preconditioner chain: a row of factor value pointers
// (forward order for P x, transposed order for P^T x) applied first to last.
// Slots are filled and retired between iteration segments, so the same batch
// serves both a whole multi-shift solve and a stream of requests.
#pragma once

#include "common.h"

struct ColInfo {
  double sigma;
  double nb, nc;      // norms of the primal and dual right-hand sides
  double tol;
  double rho, rho_prev, alpha, beta, delta;
  double rr, rtrt;    // squared norms of the current residuals
  double relp, reld;  // true relative residuals at the last check
  const double* bsrc;  // primal right-hand side (dev)
  const double* csrc;  // dual (or shadow) right-hand side (dev)
  double* xout;        // output columns (dev) or null
  double* yout;
  int32_t state, L, first, it_cycle, iters, restarts, max_restarts, maxit;
  int32_t check_p, check_d, broke, status;
  int32_t out_x, out_y;  // 0: write zeros, 1: primal iterate, 2: dual iterate
  int32_t pad0, pad1;
};

struct TraceState;

struct KrylovBatch {
  morx_system sys = nullptr;
  int cap = 0;        // column slots
  int lcap = 0;       // longest chain a slot may hold
  int prec = MORX_F64;   // factor storage
  int aprec = MORX_F64;  // preconditioner apply (MORX_F64 or MORX_F32)
  int64_t ld = 0;
  DevBuf vec, avec, cols, part, ftab;
  DevBuf plan;  // work lists of the chain steps (device-built each iteration)
  // chain grid sized from the slots' chain lengths (a batch whose columns are
  // fixed for its lifetime); otherwise from the slot count
  bool profile_grid = false;
  ColInfo* hcols = nullptr;     // pinned host mirror of the slots
  const void** hftab = nullptr;  // pinned host mirror: [2][cap][lcap]
  // graphs of one iteration segment, cached per (chain length, segment
  // length, columns, launch shape)
  struct Seg {
    int maxL;
    int64_t key;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<Seg> graphs;
};

morx_status batch_alloc(KrylovBatch& b, morx_system sys, int cap, int lcap, int prec, int aprec,
                        hipStream_t st);
// device bytes batch_alloc takes for `cap` slots
size_t batch_bytes(morx_system sys, int cap, int aprec);
void batch_free(KrylovBatch& b);
// copy slot descriptors and factor tables (host mirrors) to the device
morx_status batch_upload(KrylovBatch& b, int first, int count, hipStream_t st);
morx_status batch_download(KrylovBatch& b, hipStream_t st);
// x = x~ = 0, r = b, r~ = c for slots in COL_INIT, which then become active
morx_status batch_launch_init(KrylovBatch& b, int nc, hipStream_t st);
// `iters` BiCG iterations over slots 0..nc-1 (graph replay when use_graph)
morx_status batch_launch_segment(KrylovBatch& b, int nc, int maxL, int iters, bool use_graph,
                                 hipStream_t st, TraceState* t);
// true residuals of stopped slots; accept / restart / fail
morx_status batch_launch_true(KrylovBatch& b, int nc, hipStream_t st);
// write iterates of the listed slots to their output pointers
morx_status batch_launch_copy_out(KrylovBatch& b, const int* slots, int count, hipStream_t st);
// factor jobs and chains of one call (policy opts.chain); see bicg.hip
struct ChainPlan {
  std::vector<FactorJob> jobs;
  std::vector<std::vector<morx_factor>> chains;  // per shift, applied first to last
  bool reuse = true;                             // Algorithm 4 (keeps a vertical chain)
};
morx_status plan_chains(morx_system sys, int nshift, const double* sigmas, const morx_opts& o,
                        std::vector<morx_factor>& fresh, ChainPlan& plan);
void commit_chains(morx_system sys, const ChainPlan& plan, const double* sigmas, int prec,
                   std::vector<morx_factor>& fresh, std::vector<morx_factor>& horizontal);
TraceState* trace_state_if_on(morx_ctx ctx);
void trace_collect_pending(TraceState* t);
