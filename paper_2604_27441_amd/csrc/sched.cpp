// Batch formation policy of the serving loop (see sched.h).
#include "sched.h"

#include <algorithm>
#include <vector>

namespace revo {

int plan_batch(const SchedJob* q, int n, int* shed_run, const SchedParams& p, int* decision) {
  for (int i = 0; i < n; ++i) decision[i] = SCHED_KEEP;
  int count = 0, tokens[2] = {0, 0};
  double units = 0.0, min_deadline = 1e300;
  std::vector<unsigned> rec_streams[2];
  auto late = [&](double u, double deadline) { return p.start_ns + 1.1 * p.ns_per_unit * u + p.margin_ns > deadline; };
  // 0 = taken or shed, 1 = does not fit, 2 = the batch is closed
  auto consider = [&](int i, bool in_order) -> int {
    const SchedJob& j = q[i];
    bool fits = true, conflict = false;
    for (int m = 0; m < 2; ++m) {
      if (j.clean[m])
        for (unsigned s : rec_streams[m])
          if (s == j.stream) conflict = true;
      if (tokens[m] + j.tokens[m] > p.cap_tokens) fits = false;
    }
    bool shed_it = false;
    if (p.shed && j.units > 0.0) {
      if (late(j.units, j.deadline_ns)) {
        shed_it = true;
      } else if (count > 0 && late(units + j.units, std::min(min_deadline, j.deadline_ns))) {
        return in_order ? 2 : 1;
      }
    }
    if (count > 0 && (conflict || (!fits && !shed_it))) return in_order ? 2 : 1;
    ++count;
    if (shed_it) {
      decision[i] = SCHED_SHED;
      ++shed_run[j.stream];
      return 0;
    }
    decision[i] = SCHED_TAKE;
    for (int m = 0; m < 2; ++m) {
      tokens[m] += j.tokens[m];
      if (j.tokens[m] > 0) rec_streams[m].push_back(j.stream);
    }
    if (j.units > 0.0) {
      units += j.units;
      min_deadline = std::min(min_deadline, j.deadline_ns);
      shed_run[j.stream] = 0;
    }
    return 0;
  };
  if (p.shed) {
    // recoveries of starving streams first
    std::vector<char> seen(p.max_streams, 0);
    for (int i = 0; i < n && count < p.max_batch; ++i) {
      const unsigned s = q[i].stream;
      const bool first = !seen[s];
      seen[s] = 1;
      if (first && q[i].units > 0.0 && shed_run[s] >= p.fair_run && consider(i, false) == 2) break;
    }
  }
  for (int i = 0; i < n && count < p.max_batch; ++i) {
    if (decision[i] != SCHED_KEEP) continue;
    if (consider(i, true) == 2) break;
  }
  return count;
}

}  // namespace revo
