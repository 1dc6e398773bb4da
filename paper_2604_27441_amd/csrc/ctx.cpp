// Serving context behind revo_recover_create/submit/poll/destroy.
//
// submit() stages the caller's frames in device memory and queues a job;
// one worker thread forms batches from the queue as the GPU frees up
// (continuous batching: whatever arrived while the previous batch ran goes
// into the next one, up to the token capacity of the workspaces), applies
// clean frames to the per-stream reference rings in submission order, runs
// the RGB and depth networks on two streams, and posts completions that
// poll() hands out.  Deadlines follow the receiver's 1/fps budget (Sec. 3.3,
// Eq. 1); with shedding enabled a job that cannot finish in time completes
// as REVO_SHED, the analogue of the display repeating its last frame.  A
// stream whose recent recoveries were all shed is served first, so no stream
// is left frozen on its last good frame for a whole GoP (Sec. 3.3).
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/revo.h"
#include "model.h"
#include "sched.h"

using namespace revo;

namespace {

long long now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (long long)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

// Size-bucketed cache of device allocations, accounted against a budget.
class DevPool {
 public:
  size_t budget = 0;   // 0 = unlimited
  size_t fixed = 0;    // weights + workspaces, charged once
  size_t live = 0;     // bytes handed out or cached
  std::mutex mu;
  std::multimap<size_t, void*> free_;

  static size_t round(size_t n) { return (n + 4095) & ~(size_t)4095; }

  void* get(size_t n) {
    n = round(n);
    std::lock_guard<std::mutex> lk(mu);
    auto it = free_.find(n);
    if (it != free_.end()) {
      void* p = it->second;
      free_.erase(it);
      return p;
    }
    if (budget && fixed + live + n > budget) {
      // give back cached blocks of other sizes before refusing
      for (auto f = free_.begin(); f != free_.end() && fixed + live + n > budget;) {
        (void)hipFree(f->second);
        live -= f->first;
        f = free_.erase(f);
      }
      if (fixed + live + n > budget) return nullptr;
    }
    void* p = nullptr;
    if (hipMalloc(&p, n) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    live += n;
    return p;
  }
  void put(void* p, size_t n) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu);
    free_.emplace(round(n), p);
  }
  void clear() {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& f : free_) (void)hipFree(f.second);
    free_.clear();
  }
};

struct RefFrame {
  void* dev = nullptr;
  long long index = 0;
};

struct Ring {
  int H = 0, W = 0;
  std::deque<RefFrame> frames;  // oldest first, at most k
};

struct Mod {
  bool present = false, clean = false;
  int H = 0, W = 0;
  void* staged = nullptr;      // received frame (device, library-owned)
  uint8_t* mask = nullptr;     // loss mask (device, library-owned)
  void* out_i = nullptr;       // caller output
  float* out_f = nullptr;
  bool out_dev = false;
  void* out_i_st = nullptr;    // device staging of host outputs
  float* out_f_st = nullptr;
  float* pred = nullptr;
  size_t frame_bytes = 0;
  int error = 0;
};

struct Job {
  unsigned long long ticket = 0;
  unsigned stream = 0;
  long long frame = 0;
  unsigned flags = 0;
  long long deadline = 0, submit_ns = 0;
  Mod mod[2];
  int status = REVO_DONE, error = 0;
};

}  // namespace

namespace {
struct InFlight;
}
typedef InFlight* InFlightPtr;

struct revo_ctx {
  revo_config cfg;
  int T = 2, k = 5, J = 3, nframes = 6;
  Prec prec = P_BF16;
  ModelW model[2];
  Workspace ws[2];
  hipStream_t stream[2] = {nullptr, nullptr};
  hipStream_t copy = nullptr;
  std::mutex copy_mu;
  DevPool pool;
  std::vector<Ring> rings[2];

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::deque<revo_completion> done;
  bool stop = false;
  std::atomic<unsigned long long> next_ticket{1};
  std::thread worker, completer;
  std::deque<InFlightPtr> inflight;          // batches on the GPU, oldest first
  std::vector<int> free_slots;               // host descriptor slots not in flight
  std::condition_variable cv_inflight;
  bool completer_stop = false;
  int inflight_max = 2;
  bool use_graphs = false;
  std::atomic<bool> calibrating{false};
  std::mutex calib_mu;
  hipEvent_t done_ev[WS_SLOTS][2] = {};
  hipStream_t d2h = nullptr;
  double busy_until_ns = 0.0;  // when the GPU is expected to drain what is enqueued (guarded by mu)
  long long last_done_ns = 0;
  int device_error = 0;
  double sec_per_unit = 3e-11;  // cost model for shedding: seconds per work unit (guarded by mu)
  // completion time minus predicted completion of recent batches (ns,
  // guarded by mu): its tail widens the shedding margin
  std::vector<double> lateness;
  size_t lateness_next = 0;
  // per stream (guarded by mu): frame size of the last clean frame submitted
  // per modality (a recovery needs one at its own size), and the run of
  // recoveries shed since the last one admitted to a batch (sched.h)
  struct StreamState {
    int clean_h[2] = {0, 0}, clean_w[2] = {0, 0};
  };
  std::vector<StreamState> sst;
  std::vector<int> shed_run;
  // reference frames dropped by a resolution change while batches launched
  // before it may still read them: returned to the pool once every batch
  // numbered below `after` has completed (guarded by mu)
  struct Deferred {
    void* p;
    size_t n;
    unsigned long long after;
  };
  std::vector<Deferred> deferred;
  unsigned long long batch_seq = 0;       // batches formed so far (guarded by mu)
  unsigned long long completed_seq = 0;   // every batch up to this number has completed (guarded by mu)
  hipEvent_t caller_ev = nullptr;         // orders input copies after cfg.hip_stream (guarded by copy_mu)
  std::mutex stats_mu;
  revo_stats stats;
};

namespace {

const int kMaxQueue = 4096;
// Shedding policy (sched.h): a stream whose last kFairRun recovery requests
// were all shed goes ahead of the submission order (half of a 30-frame GoP, so
// every stream keeps a served recovery in every GoP-long window while the GPU
// can afford one per stream per kFairRun frames).
const int kFairRun = 15;

// Shedding margin: 3 ms, or the 99th percentile of how late the last
// kLatenessWindow batches completed against their prediction plus 1 ms,
// whichever is larger (at most 10 ms).
const size_t kLatenessWindow = 256;

double shed_margin_ns(const std::vector<double>& late) {
  if (late.size() < 16) return 3e6;
  std::vector<double> v(late);
  const size_t k = (v.size() * 99) / 100;
  std::nth_element(v.begin(), v.begin() + k, v.end());
  return std::min(10e6, std::max(3e6, v[k] + 1e6));
}

void release_mod(revo_ctx* c, Mod& m, int C) {
  const size_t px = (size_t)m.H * m.W;
  if (m.staged) c->pool.put(m.staged, m.frame_bytes);
  if (m.mask) c->pool.put(m.mask, px);
  if (m.pred) c->pool.put(m.pred, px * C * 4);
  if (m.out_i_st) c->pool.put(m.out_i_st, m.frame_bytes);
  if (m.out_f_st) c->pool.put(m.out_f_st, px * C * 4);
  m.staged = nullptr; m.mask = nullptr; m.pred = nullptr; m.out_i_st = nullptr; m.out_f_st = nullptr;
}

void finish(revo_ctx* c, Job* j) {
  for (int q = 0; q < 2; ++q) release_mod(c, j->mod[q], q == 0 ? 3 : 1);
  revo_completion rc;
  rc.ticket = j->ticket;
  rc.stream_id = j->stream;
  rc.frame_index = j->frame;
  rc.status = j->status;
  rc.error = j->error;
  rc.submit_ns = j->submit_ns;
  rc.done_ns = now_ns();
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->done.push_back(rc);
  }
  c->cv_done.notify_all();
  delete j;
}

// Return reference frames dropped by batch `seq` to the pool once every
// earlier batch has completed (they may still be reading them).
void defer_free(revo_ctx* c, void* p, size_t n, unsigned long long seq) {
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->completed_seq + 1 < seq) {
      c->deferred.push_back({p, n, seq});
      return;
    }
  }
  c->pool.put(p, n);
}

// Push a clean frame into its stream's ring on the modality's stream (the
// ring slot is only read by batches launched earlier on that same stream).
// seq numbers the batch being formed.
int push_clean(revo_ctx* c, Job* j, int q, unsigned long long seq) {
  Mod& m = j->mod[q];
  Ring& ring = c->rings[q][j->stream];
  if (ring.H != m.H || ring.W != m.W) {
    // a resolution change starts a new reference set; the old frames may
    // still be read by batches in flight, so their memory waits for them
    for (auto& f : ring.frames) defer_free(c, f.dev, (size_t)ring.H * ring.W * (q == 0 ? 3 : 2), seq);
    ring.frames.clear();
    ring.H = m.H; ring.W = m.W;
  }
  RefFrame slot;
  if ((int)ring.frames.size() >= c->k) {
    slot = ring.frames.front();
    ring.frames.pop_front();
  } else {
    slot.dev = c->pool.get(m.frame_bytes);
    if (!slot.dev) return REVO_ENOMEM;
  }
  if (hipMemcpyAsync(slot.dev, m.staged, m.frame_bytes, hipMemcpyDeviceToDevice, c->stream[q]) != hipSuccess)
    return REVO_EDEVICE;
  slot.index = j->frame;
  ring.frames.push_back(slot);
  return 0;
}

// Fill one kernel descriptor for modality q of job j.
void fill_desc(revo_ctx* c, Job* j, int q, ReqDesc& d) {
  Mod& m = j->mod[q];
  memset(&d, 0, sizeof(d));
  d.H = m.H; d.W = m.W;
  d.mask = m.clean ? nullptr : m.mask;
  d.pred = m.pred;
  d.out_i = m.out_dev ? m.out_i : m.out_i_st;
  d.out_f = m.out_dev ? m.out_f : m.out_f_st;
  if (m.clean) {
    d.J = 1; d.nframes = 1;
    d.frames[0] = m.staged;
    return;
  }
  // frames: k references oldest first (the oldest repeated when fewer are
  // held), padded at the old end to a multiple of T, then the target
  const Ring& ring = c->rings[q][j->stream];
  const int have = (int)ring.frames.size();
  std::vector<RefFrame> seq;
  for (int i = 0; i < c->k - have; ++i) seq.push_back(ring.frames.front());
  for (const RefFrame& f : ring.frames) seq.push_back(f);
  RefFrame tgt;
  tgt.dev = m.staged;
  tgt.index = j->frame;
  seq.push_back(tgt);
  while ((int)seq.size() % c->T) seq.insert(seq.begin(), seq.front());
  d.nframes = (int)seq.size();
  d.J = d.nframes / c->T;
  for (int i = 0; i < d.nframes; ++i) d.frames[i] = seq[i].dev;
  for (int jj = 0; jj < d.J; ++jj) d.tau[jj] = (float)(j->frame - seq[jj * c->T].index);
}

// A batch enqueued on the GPU, waiting for its completion events.
struct InFlight {
  std::vector<Job*> batch;
  unsigned long long seq = 0;  // batch number (batches complete in this order)
  bool record = false;  // FP8 calibration batch
  int slot = 0;
  int rc = 0;
  double units = 0.0;
  long long t_enq = 0;
  double predicted_done_ns = 0.0;
};

// Enqueue one batch (descriptors in host slot `slot`) on the modality streams
// and record its completion events.
int launch_batch(revo_ctx* c, InFlight* f) {
  std::vector<std::pair<Job*, int>> rec[2], cln[2];
  for (Job* j : f->batch) {
    if (j->status != REVO_DONE) continue;
    for (int q = 0; q < 2; ++q) {
      Mod& m = j->mod[q];
      if (!m.present || m.error) continue;
      (m.clean ? cln[q] : rec[q]).push_back({j, q});
    }
  }
  int rc = 0;
  for (int q = 0; q < 2; ++q) {
    Workspace& w = c->ws[q];
    ReqDesc* hr = w.h_reqs_slot[f->slot];
    int n = 0;
    for (auto& e : rec[q]) fill_desc(c, e.first, q, hr[n++]);
    const int nrec = n;
    for (auto& e : cln[q]) fill_desc(c, e.first, q, hr[n++]);
    if (n == 0) continue;
    const int e = forward(c->model[q], w, f->slot, nrec, n, c->cfg.composite, c->use_graphs, c->stream[q], f->record);
    if (e) rc = e;
  }
  for (int q = 0; q < 2; ++q)
    if (hipEventRecord(c->done_ev[f->slot][q], c->stream[q]) != hipSuccess) rc = REVO_EDEVICE;
  return rc;
}

// Wait for a batch, copy host outputs, post its completions.
void complete_batch(revo_ctx* c, InFlight* f) {
  int rc = f->rc;
  for (int q = 0; q < 2; ++q)
    if (hipEventSynchronize(c->done_ev[f->slot][q]) != hipSuccess) rc = REVO_EDEVICE;
  for (Job* j : f->batch) {
    if (j->status != REVO_DONE || rc) continue;
    for (int q = 0; q < 2; ++q) {
      Mod& m = j->mod[q];
      if (!m.present || m.error || m.out_dev) continue;
      const size_t px = (size_t)m.H * m.W;
      if (m.out_i && hipMemcpyAsync(m.out_i, m.out_i_st, m.frame_bytes, hipMemcpyDeviceToHost, c->d2h) != hipSuccess)
        rc = REVO_EDEVICE;
      if (m.out_f &&
          hipMemcpyAsync(m.out_f, m.out_f_st, px * (q == 0 ? 3 : 1) * 4, hipMemcpyDeviceToHost, c->d2h) != hipSuccess)
        rc = REVO_EDEVICE;
    }
  }
  if (hipStreamSynchronize(c->d2h) != hipSuccess) rc = REVO_EDEVICE;
  {
    // GPU span of this batch: from its enqueue or the previous completion,
    // whichever is later; it refines the cost model and the drain estimate
    std::lock_guard<std::mutex> lk(c->mu);
    const long long t_done = now_ns();
    const double span = (double)(t_done - std::max(f->t_enq, c->last_done_ns)) * 1e-9;
    if (f->units > 0.0 && rc == 0 && span > 0.0) c->sec_per_unit = 0.7 * c->sec_per_unit + 0.3 * (span / f->units);
    c->last_done_ns = t_done;
    if (f->units > 0.0 && rc == 0) {
      const double late = (double)t_done - f->predicted_done_ns;
      if (c->lateness.size() < kLatenessWindow) c->lateness.push_back(late);
      else c->lateness[c->lateness_next++ % kLatenessWindow] = late;
    }
    if (c->inflight.size() > 1) c->busy_until_ns += (double)t_done - f->predicted_done_ns;
    else c->busy_until_ns = (double)t_done;
  }
  if (rc) {
    c->device_error = rc;
    for (Job* j : f->batch)
      if (j->status == REVO_DONE) { j->status = REVO_FAILED; j->error = rc; }
  }
  {
    std::lock_guard<std::mutex> lk(c->stats_mu);
    revo_stats& st = c->stats;
    st.batches += 1;
    for (Job* j : f->batch) {
      if (j->status == REVO_DONE) st.served++;
      else if (j->status == REVO_SHED) st.shed++;
      else st.failed++;
    }
    for (int q = 0; q < 2; ++q) {
      Prof& p = c->ws[q].prof;
      if (!p.on) continue;
      if (rc == 0) (void)prof_collect(p);
      p.recs.clear();
      p.used = 0;
      st.attn_launches += p.count[PK_ATTN]; st.attn_ms += p.ms[PK_ATTN]; st.attn_flop += p.flop[PK_ATTN];
      st.gemm_launches += p.count[PK_GEMM]; st.gemm_ms += p.ms[PK_GEMM]; st.gemm_flop += p.flop[PK_GEMM];
      st.other_launches += p.count[PK_OTHER]; st.other_ms += p.ms[PK_OTHER];
      st.forward_ms += p.ms[PK_FORWARD];
      for (int k = 0; k < PK_N; ++k) { p.ms[k] = 0; p.flop[k] = 0; p.count[k] = 0; }
    }
  }
  for (Job* j : f->batch) finish(c, j);
}

void completer_main(revo_ctx* c) {
  (void)hipSetDevice(c->cfg.device);
  for (;;) {
    InFlight* f = nullptr;
    {
      std::unique_lock<std::mutex> lk(c->mu);
      c->cv_inflight.wait(lk, [&] { return !c->inflight.empty() || c->completer_stop; });
      if (c->inflight.empty()) return;
      f = c->inflight.front();
    }
    complete_batch(c, f);
    std::vector<revo_ctx::Deferred> ready;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      c->inflight.pop_front();
      c->free_slots.push_back(f->slot);
      c->completed_seq = f->seq;
      auto& dl = c->deferred;
      for (size_t i = 0; i < dl.size();) {
        if (dl[i].after <= f->seq + 1) {
          ready.push_back(dl[i]);
          dl[i] = dl.back();
          dl.pop_back();
        } else {
          ++i;
        }
      }
    }
    for (auto& d : ready) c->pool.put(d.p, d.n);
    c->cv_work.notify_all();
    c->cv_done.notify_all();
    delete f;
  }
}

void worker_main(revo_ctx* c) {
  (void)hipSetDevice(c->cfg.device);
  const int cap = c->cfg.max_batch_tokens;
  const int max_batch = c->cfg.max_batch;
  for (;;) {
    std::vector<Job*> batch;
    int slot = -1;
    unsigned long long seq = 0;
    double batch_start = 0.0;
    {
      std::unique_lock<std::mutex> lk(c->mu);
      for (;;) {
        if (c->stop && c->queue.empty()) return;
        if (!c->queue.empty() && !c->free_slots.empty()) {
          bool release = c->stop;
          for (Job* j : c->queue)
            if (!(j->flags & REVO_HOLD)) { release = true; break; }
          if (!release && now_ns() - c->queue.front()->submit_ns > 2000000LL) release = true;
          if (release) break;
          c->cv_work.wait_for(lk, std::chrono::microseconds(500));
          continue;
        }
        c->cv_work.wait(lk);
      }
      slot = c->free_slots.back();
      c->free_slots.pop_back();
      // the next batch (sched.h): submission order, starving streams first,
      // deadline shedding
      const int nq = (int)c->queue.size();
      std::vector<SchedJob> sj(nq);
      std::vector<int> dec(nq);
      for (int i = 0; i < nq; ++i) {
        const Job* j = c->queue[i];
        SchedJob& e = sj[i];
        e.stream = j->stream;
        e.units = 0.0;
        e.deadline_ns = (double)j->deadline;
        for (int q = 0; q < 2; ++q) {
          const Mod& m = j->mod[q];
          e.clean[q] = m.present && m.clean;
          e.tokens[q] = 0;
          if (m.present && !m.clean) {
            const int N = request_tokens(m.H, m.W, c->J);
            const int al = c->cfg.precision == REVO_FP8 ? 64 : 16;  // rows start on a V^T key group
            e.tokens[q] = (N + al - 1) / al * al;
            e.units += work_units(N);
          }
        }
      }
      SchedParams sp;
      sp.shed = (c->cfg.flags & REVO_CFG_SHED) != 0;
      sp.start_ns = std::max((double)now_ns(), c->busy_until_ns);
      sp.ns_per_unit = 1e9 * c->sec_per_unit;
      sp.cap_tokens = cap;
      sp.max_batch = max_batch;
      sp.fair_run = kFairRun;
      sp.max_streams = c->cfg.max_streams;
      sp.margin_ns = shed_margin_ns(c->lateness);
      plan_batch(sj.data(), nq, c->shed_run.data(), sp, dec.data());
      const double start = sp.start_ns;
      // the batch in submission order, as the ring updates below expect; the
      // rest stays queued in order
      {
        std::deque<Job*> rest;
        for (int i = 0; i < nq; ++i) {
          Job* j = c->queue[i];
          if (dec[i] == SCHED_KEEP) {
            rest.push_back(j);
            continue;
          }
          if (dec[i] == SCHED_SHED) j->status = REVO_SHED;
          batch.push_back(j);
        }
        c->queue.swap(rest);
      }
      batch_start = start;
      seq = ++c->batch_seq;
    }
    c->cv_done.notify_all();  // queue space freed

    // ring updates and reference checks in submission order
    const long long t0 = now_ns();
    const double start = batch_start;
    double units = 0.0;
    for (Job* j : batch) {
      double ju = 0.0;
      for (int q = 0; q < 2; ++q)
        if (j->mod[q].present && !j->mod[q].clean) ju += work_units(request_tokens(j->mod[q].H, j->mod[q].W, c->J));
      if (j->status == REVO_DONE) units += ju;
      for (int q = 0; q < 2; ++q) {
        Mod& m = j->mod[q];
        if (!m.present) continue;
        if (m.clean) {
          // clean frames always refresh the references, shed or not
          const int e = push_clean(c, j, q, seq);
          if (e) { m.error = e; j->status = REVO_FAILED; j->error = e; }
        } else if (j->status == REVO_DONE) {
          // (submit checked that a clean frame of this size came first; its
          // ring update can still have failed for memory)
          const Ring& ring = c->rings[q][j->stream];
          if (ring.frames.empty() || ring.H != m.H || ring.W != m.W) {
            m.error = REVO_ENOREF; j->status = REVO_FAILED; j->error = REVO_ENOREF;
          }
        }
      }
    }
    InFlight* f = new InFlight();
    f->batch.swap(batch);
    f->seq = seq;
    f->record = c->calibrating.load();
    f->slot = slot;
    f->units = units;
    f->t_enq = t0;
    f->rc = launch_batch(c, f);
    {
      std::lock_guard<std::mutex> lk(c->mu);
      c->busy_until_ns = std::max(start, c->busy_until_ns) + 1e9 * c->sec_per_unit * units;
      f->predicted_done_ns = c->busy_until_ns;
      c->inflight.push_back(f);
    }
    c->cv_inflight.notify_all();
  }
}

int stage_mod(revo_ctx* c, Mod& m, const void* frame, const unsigned char* mask, void* out_i, float* out_f,
              int C, int H, int W, bool dev) {
  const size_t px = (size_t)H * W;
  m.present = true;
  m.clean = (mask == nullptr);
  m.H = H; m.W = W;
  m.frame_bytes = px * (C == 3 ? 3 : 2);
  m.out_i = out_i; m.out_f = out_f; m.out_dev = dev;
  m.staged = c->pool.get(m.frame_bytes);
  if (!m.staged) return REVO_EAGAIN;
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (hipMemcpyAsync(m.staged, frame, m.frame_bytes, kind, c->copy) != hipSuccess) return REVO_EDEVICE;
  if (!m.clean) {
    m.mask = (uint8_t*)c->pool.get(px);
    if (!m.mask) return REVO_EAGAIN;
    if (hipMemcpyAsync(m.mask, mask, px, kind, c->copy) != hipSuccess) return REVO_EDEVICE;
    // the prediction buffer is admitted here too, so that a queued job never
    // fails for memory later
    m.pred = (float*)c->pool.get(px * C * 4);
    if (!m.pred) return REVO_EAGAIN;
  }
  if (!dev) {
    if (out_i && !(m.out_i_st = c->pool.get(m.frame_bytes))) return REVO_EAGAIN;
    if (out_f && !(m.out_f_st = (float*)c->pool.get(px * C * 4))) return REVO_EAGAIN;
  }
  return 0;
}

}  // namespace

extern "C" {

void revo_config_default(revo_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->precision = REVO_BF16;
  cfg->k = 5;
  cfg->tubelet = 2;
  cfg->composite = 1;
  cfg->fps = 30.0f;
}

size_t revo_weight_count(int channels, int tubelet, int enc_depth, int dec_depth) {
  if ((channels != 1 && channels != 3) || tubelet < 1 || enc_depth < 0 || dec_depth < 0) return 0;
  return weight_count(channels, tubelet, enc_depth, dec_depth);
}

const char* revo_strerror(int code) {
  switch (code) {
    case REVO_OK: return "ok";
    case REVO_EAGAIN: return "queue or staging full, poll and retry";
    case REVO_EINVAL: return "invalid argument";
    case REVO_ENOMEM: return "out of device memory or HBM budget";
    case REVO_EDEVICE: return "HIP device error";
    case REVO_ENOREF: return "no clean reference frame for this stream";
    case REVO_ENOTSUP: return "unsupported configuration";
    case REVO_ESHUTDOWN: return "context shutting down";
    case REVO_E2BIG: return "size beyond the fixed workspace";
  }
  return "unknown error";
}

int revo_recover_create(const revo_config* cfg_in, revo_ctx** out) {
  if (!cfg_in || !out) return REVO_EINVAL;
  *out = nullptr;
  revo_config cfg = *cfg_in;
  if (cfg.precision != REVO_FP32 && cfg.precision != REVO_BF16 && cfg.precision != REVO_FP8) return REVO_ENOTSUP;
  if (cfg.k < 1 || cfg.k > 7 || cfg.tubelet < 1 || cfg.tubelet > 4) return REVO_EINVAL;
  const int T = cfg.tubelet;
  const int nframes = (cfg.k + 1 + T - 1) / T * T;
  if (nframes > REVO_MAX_FRAMES) return REVO_ENOTSUP;
  if (cfg.enc_depth == 0) cfg.enc_depth = 12;
  if (cfg.dec_depth == 0) cfg.dec_depth = 4;
  if (cfg.enc_depth < 0 || cfg.dec_depth < 0 || cfg.enc_depth > 64 || cfg.dec_depth > 64) return REVO_EINVAL;
  if (cfg.max_streams <= 0) cfg.max_streams = 64;
  if (cfg.max_batch <= 0) cfg.max_batch = 16;
  if (cfg.fps <= 0.0f) cfg.fps = 30.0f;
  if (!cfg.weights_rgb || !cfg.weights_depth) return REVO_EINVAL;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || cfg.device < 0 || cfg.device >= ndev) return REVO_EDEVICE;
  if (hipSetDevice(cfg.device) != hipSuccess) return REVO_EDEVICE;

  revo_ctx* c = new revo_ctx();
  memset(&c->stats, 0, sizeof(c->stats));
  c->cfg = cfg;
  c->T = T; c->k = cfg.k; c->nframes = nframes; c->J = nframes / T;
  c->prec = cfg.precision == REVO_BF16 ? P_BF16 : cfg.precision == REVO_FP8 ? P_FP8 : P_FP32;
  c->rings[0].resize(cfg.max_streams);
  c->rings[1].resize(cfg.max_streams);
  c->sst.resize(cfg.max_streams);
  c->shed_run.assign(cfg.max_streams, 0);
  int rc = 0;
  const int nstreams = (cfg.flags & REVO_CFG_ONE_STREAM) ? 1 : 2;
  for (int q = 0; q < nstreams && !rc; ++q)
    if (hipStreamCreateWithFlags(&c->stream[q], hipStreamNonBlocking) != hipSuccess) rc = REVO_EDEVICE;
  if (nstreams == 1) c->stream[1] = c->stream[0];
  if (!rc && hipStreamCreateWithFlags(&c->copy, hipStreamNonBlocking) != hipSuccess) rc = REVO_EDEVICE;
  if (!rc && hipStreamCreateWithFlags(&c->d2h, hipStreamNonBlocking) != hipSuccess) rc = REVO_EDEVICE;
  if (!rc && cfg.hip_stream && hipEventCreateWithFlags(&c->caller_ev, hipEventDisableTiming) != hipSuccess)
    rc = REVO_EDEVICE;
  for (int sl = 0; sl < WS_SLOTS && !rc; ++sl)
    for (int q = 0; q < 2 && !rc; ++q)
      if (hipEventCreateWithFlags(&c->done_ev[sl][q], hipEventDisableTiming) != hipSuccess) rc = REVO_EDEVICE;
  if (!rc) rc = model_load(c->model[0], 3, T, cfg.enc_depth, cfg.dec_depth, c->prec, cfg.weights_rgb, cfg.n_weights_rgb, c->stream[0]);
  if (!rc) rc = model_load(c->model[1], 1, T, cfg.enc_depth, cfg.dec_depth, c->prec, cfg.weights_depth, cfg.n_weights_depth, c->stream[1]);
  if (!rc) {
    size_t fixed = c->model[0].bytes + c->model[1].bytes;
    int cap = cfg.max_batch_tokens;
    if (cap <= 0) {
      cap = 43200;
      if (cfg.hbm_budget_bytes) {
        // largest capacity whose two workspaces leave a quarter of the budget for rings and staging
        const double per_tok = (double)(workspace_bytes(c->model[0], 1 << 16, cfg.max_batch) +
                                        workspace_bytes(c->model[1], 1 << 16, cfg.max_batch)) / (1 << 16);
        const double avail = 0.75 * (double)cfg.hbm_budget_bytes - (double)fixed;
        cap = avail > 0 ? (int)std::min(avail / per_tok, 1.0e6) : 0;
      }
    }
    cap &= ~15;  // requests start on 16-row boundaries (V^T key groups of 16)
    if (cap < 64) rc = REVO_ENOMEM;
    c->cfg.max_batch_tokens = cap;
    if (!rc) rc = workspace_alloc(c->ws[0], c->model[0], cap, cfg.max_batch, c->stream[0]);
    if (!rc) rc = workspace_alloc(c->ws[1], c->model[1], cap, cfg.max_batch, c->stream[1]);
    if (!rc && (cfg.flags & (REVO_CFG_PROFILE | REVO_CFG_PROFILE_ATTN)))
      for (int q = 0; q < 2 && !rc; ++q) {
        rc = prof_init(c->ws[q].prof, 1024);
        c->ws[q].prof.attn_only = !(cfg.flags & REVO_CFG_PROFILE);
      }
    fixed += c->ws[0].bytes + c->ws[1].bytes;
    c->pool.fixed = fixed;
    c->pool.budget = cfg.hbm_budget_bytes;
    if (!rc && cfg.hbm_budget_bytes && fixed > cfg.hbm_budget_bytes) rc = REVO_ENOMEM;
  }
  if (rc) {
    revo_recover_destroy(c);
    return rc < 0 ? rc : REVO_EDEVICE;
  }
  // event records are per workspace
  c->inflight_max = (cfg.flags & (REVO_CFG_PROFILE | REVO_CFG_PROFILE_ATTN)) ? 1 : WS_SLOTS;
  c->use_graphs = (cfg.flags & REVO_CFG_GRAPHS) != 0;
  for (int sl = 0; sl < c->inflight_max; ++sl) c->free_slots.push_back(sl);
  c->worker = std::thread(worker_main, c);
  c->completer = std::thread(completer_main, c);
  *out = c;
  return REVO_OK;
}

int revo_recover_submit(revo_ctx* c, const revo_request* r, unsigned long long* ticket) {
  if (!c || !r) return REVO_EINVAL;
  if (r->stream_id >= (unsigned)c->cfg.max_streams) return REVO_EINVAL;
  if (r->width < 16 || r->height < 16 || r->width > 4096 || r->height > 4096) return REVO_EINVAL;
  if (!r->rgb && !r->depth) return REVO_EINVAL;
  if ((r->mask_rgb && !r->rgb) || (r->mask_depth && !r->depth)) return REVO_EINVAL;
  {
    const int al = c->cfg.precision == REVO_FP8 ? 64 : 16;
    if ((request_tokens(r->height, r->width, c->J) + al - 1) / al * al > c->cfg.max_batch_tokens) return REVO_EINVAL;
  }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->stop) return REVO_ESHUTDOWN;
    if ((int)c->queue.size() >= kMaxQueue) return REVO_EAGAIN;
  }
  const bool dev = (r->flags & REVO_DEVICE_PTRS) != 0;
  if (dev) {
    // every device pointer must belong to the device (host memory would fault the kernels)
    const void* ptrs[] = {r->rgb, r->mask_rgb, r->depth, r->mask_depth, r->rgb_out, r->depth_out, r->rgb_out_f32,
                          r->depth_out_f32};
    for (const void* p : ptrs)
      if (p && !is_device_ptr(p)) return REVO_EINVAL;
  }
  Job* j = new Job();
  j->stream = r->stream_id;
  j->frame = r->frame_index;
  j->flags = r->flags;
  j->submit_ns = now_ns();
  j->deadline = r->deadline_ns ? r->deadline_ns : j->submit_ns + (long long)(1e9 / c->cfg.fps);
  int rc = 0;
  {
    std::lock_guard<std::mutex> lk(c->copy_mu);
    (void)hipSetDevice(c->cfg.device);
    // the input copies come after the caller's work already on its stream
    if (c->caller_ev && (hipEventRecord(c->caller_ev, (hipStream_t)c->cfg.hip_stream) != hipSuccess ||
                         hipStreamWaitEvent(c->copy, c->caller_ev, 0) != hipSuccess))
      rc = REVO_EDEVICE;
    if (!rc && r->rgb) rc = stage_mod(c, j->mod[0], r->rgb, r->mask_rgb, r->rgb_out, r->rgb_out_f32, 3, r->height, r->width, dev);
    if (!rc && r->depth)
      rc = stage_mod(c, j->mod[1], r->depth, r->mask_depth, r->depth_out, r->depth_out_f32, 1, r->height, r->width, dev);
    if (hipStreamSynchronize(c->copy) != hipSuccess && !rc) rc = REVO_EDEVICE;
  }
  if (rc) {
    for (int q = 0; q < 2; ++q) release_mod(c, j->mod[q], q == 0 ? 3 : 1);
    delete j;
    return rc;
  }
  {
    // A recovery needs a clean frame of its stream and modality at its own
    // size submitted before it (Sec. 3.4.1: the k closest clean frames are
    // its input); a clean frame becomes that stream's reference.  Checked in
    // queue order, so tickets follow the queue.
    std::lock_guard<std::mutex> lk(c->mu);
    revo_ctx::StreamState& ss = c->sst[j->stream];
    for (int q = 0; q < 2 && !rc; ++q) {
      const Mod& m = j->mod[q];
      if (m.present && !m.clean && (ss.clean_h[q] != m.H || ss.clean_w[q] != m.W)) rc = REVO_ENOREF;
    }
    if (!rc) {
      for (int q = 0; q < 2; ++q)
        if (j->mod[q].present && j->mod[q].clean) { ss.clean_h[q] = j->mod[q].H; ss.clean_w[q] = j->mod[q].W; }
      j->ticket = c->next_ticket++;
      if (ticket) *ticket = j->ticket;
      c->queue.push_back(j);
    }
  }
  if (rc) {
    for (int q = 0; q < 2; ++q) release_mod(c, j->mod[q], q == 0 ? 3 : 1);
    delete j;
    return rc;
  }
  c->cv_work.notify_one();
  return REVO_OK;
}

int revo_recover_poll(revo_ctx* c, revo_completion* out, int max, int timeout_us) {
  if (!c || (!out && max > 0) || max < 0) return REVO_EINVAL;
  std::unique_lock<std::mutex> lk(c->mu);
  auto ready = [&] { return !c->done.empty(); };
  if (timeout_us < 0) c->cv_done.wait(lk, ready);
  else if (timeout_us > 0) c->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  int n = 0;
  while (n < max && !c->done.empty()) {
    out[n++] = c->done.front();
    c->done.pop_front();
  }
  return n;
}

int revo_calibrate(revo_ctx* c, int phase) {
  if (!c) return REVO_EINVAL;
  if (c->prec != P_FP8) return REVO_ENOTSUP;
  if (phase != 0 && phase != 1) return REVO_EINVAL;
  std::lock_guard<std::mutex> guard(c->calib_mu);
  (void)hipSetDevice(c->cfg.device);
  // let every batch formed so far finish (they ran with the previous mode)
  {
    std::unique_lock<std::mutex> lk(c->mu);
    c->cv_done.wait(lk, [&] { return (c->queue.empty() && c->inflight.empty()) || c->stop; });
    if (c->stop) return REVO_ESHUTDOWN;
    // the worker holds no batch now: change the mode before it forms the next
    int rc = 0;
    for (int q = 0; q < 2 && !rc; ++q) {
      rc = phase ? model_reset_calibration(c->model[q], c->stream[q])
                 : model_finish_calibration(c->model[q], c->stream[q]);
      // graphs captured before hold the previous mode's launches
      for (auto& g : c->ws[q].graph)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    }
    for (int q = 0; q < 2 && !rc; ++q)
      if (hipStreamSynchronize(c->stream[q]) != hipSuccess) rc = REVO_EDEVICE;
    if (rc) return rc < 0 ? rc : REVO_EDEVICE;
    c->calibrating = phase == 1;
  }
  return REVO_OK;
}

int revo_get_stats(revo_ctx* c, revo_stats* out, int reset) {
  if (!c || !out) return REVO_EINVAL;
  std::lock_guard<std::mutex> lk(c->stats_mu);
  *out = c->stats;
  if (reset) memset(&c->stats, 0, sizeof(c->stats));
  {
    std::lock_guard<std::mutex> pl(c->pool.mu);
    out->hbm_fixed_bytes = (long long)c->pool.fixed;
    out->hbm_pool_bytes = (long long)c->pool.live;
  }
  return REVO_OK;
}

void revo_recover_destroy(revo_ctx* c) {
  if (!c) return;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->stop = true;
  }
  c->cv_work.notify_all();
  if (c->worker.joinable()) c->worker.join();
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->completer_stop = true;
  }
  c->cv_inflight.notify_all();
  if (c->completer.joinable()) c->completer.join();
  (void)hipSetDevice(c->cfg.device);
  for (int q = 0; q < 2; ++q) {
    if (c->stream[q]) (void)hipStreamSynchronize(c->stream[q]);
    for (Ring& ring : c->rings[q])
      for (auto& f : ring.frames) c->pool.put(f.dev, (size_t)ring.H * ring.W * (q == 0 ? 3 : 2));
    workspace_free(c->ws[q]);
    model_free(c->model[q]);
  }
  for (auto& d : c->deferred) c->pool.put(d.p, d.n);  // every batch has completed
  c->deferred.clear();
  c->pool.clear();
  if (c->caller_ev) (void)hipEventDestroy(c->caller_ev);
  if (c->stream[0]) (void)hipStreamDestroy(c->stream[0]);
  if (c->stream[1] && c->stream[1] != c->stream[0]) (void)hipStreamDestroy(c->stream[1]);
  if (c->copy) (void)hipStreamDestroy(c->copy);
  if (c->d2h) (void)hipStreamDestroy(c->d2h);
  for (int sl = 0; sl < WS_SLOTS; ++sl)
    for (int q = 0; q < 2; ++q)
      if (c->done_ev[sl][q]) (void)hipEventDestroy(c->done_ev[sl][q]);
  delete c;
}

}  // extern "C"
