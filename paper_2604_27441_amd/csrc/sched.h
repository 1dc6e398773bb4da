// Batch formation policy of the serving loop: which queued jobs go into the
// next batch, which are shed, which wait.  Host logic only (no HIP), so that
// it can be checked on its own with a fake clock.
#pragma once

namespace revo {

struct SchedJob {
  unsigned stream;
  int tokens[2];        // token rows a recovered modality adds to the batch (0: none)
  bool clean[2];        // modality present as a clean frame (a reference update)
  double units;         // work units of the job's recoveries (0: clean frames only)
  double deadline_ns;   // CLOCK_MONOTONIC
};

struct SchedParams {
  bool shed;            // shed jobs that cannot meet their deadline
  double start_ns;      // when the batch can start on the GPU
  double ns_per_unit;   // cost model
  int cap_tokens;       // token rows per modality per batch
  int max_batch;        // jobs per batch (shed ones included)
  int fair_run;         // a stream with this many shed recoveries in a row goes first
  int max_streams;
  double margin_ns;     // fixed part of the plan's safety margin
};

enum { SCHED_KEEP = 0, SCHED_TAKE = 1, SCHED_SHED = 2 };

// Work units of a request of N tokens: attention grows as N^2, the products
// as N (the constant is the ratio of their FLOPs per token at 64-wide heads).
inline double work_units(int N) { return (double)N * N + 2300.0 * N; }

// Plan the next batch from q[0 .. n), oldest first.  decision[i] receives a
// SCHED_* value; shed_run[stream] (max_streams entries) counts the recoveries
// of each stream shed in a row and is updated.  Returns how many jobs leave
// the queue (taken or shed).
//
// Jobs are taken in submission order while they fit, except that a recovery
// of a stream with at least fair_run shed recoveries in a row goes first when
// no earlier job of its stream is queued (reference updates must reach the
// ring in submission order).  The submission-order pass stops at the first
// job that does not fit, and before a clean frame of a stream that already
// has a recovery in the batch.  With shedding, a job that would miss its
// deadline even alone, started at start_ns, is shed; the batch, which
// completes at once, closes before a job that would make a member miss its
// deadline.  The plan keeps a margin of
// margin_ns (completion hand-off and output copies after the GPU span, and
// the cost model's recent tail error) plus 10 % of the predicted cost.
int plan_batch(const SchedJob* q, int n, int* shed_run, const SchedParams& p, int* decision);

}  // namespace revo
