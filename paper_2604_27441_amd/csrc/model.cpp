// Weights upload, workspace sizing and the launch sequence of the recovery
// network (Sec. 3.4.1: tubelet embedding, encoder, decoder over all tokens,
// reconstruction of the target frame; App. B.1: no token shuffling).
#include "model.h"

#include <string.h>

namespace revo {

namespace {

// bytes of a BF16-level operand (the FP8 form keeps BF16 copies and buffers)
size_t esize(Prec p) { return p == P_FP32 ? 4 : 2; }
Prec base_prec(Prec p) { return p == P_FP32 ? P_FP32 : P_BF16; }

size_t block_count(int D) { return 2 * D + 3 * D * D + 3 * D + D * D + D + 2 * D + 4 * D * D + 4 * D + 4 * D * D + D; }

}  // namespace

size_t weight_count(int C, int T, int ne, int nd) {
  const size_t L = (size_t)T * 256 * C;
  const size_t De = 384, Dd = 192;
  return De * L + De + ne * block_count(De) + 2 * De + Dd * De + Dd + nd * block_count(Dd) + 2 * Dd + L * Dd + L;
}

int model_load(ModelW& m, int C, int T, int ne, int nd, Prec p, const float* host_blob, size_t n, hipStream_t s) {
  m.C = C; m.T = T; m.ne = ne; m.nd = nd; m.prec = p;
  m.count = weight_count(C, T, ne, nd);
  if (n != m.count || !host_blob) return -22;
  REVO_HIP_TRY(hipMalloc(&m.master, m.count * 4));
  REVO_HIP_TRY(hipMemcpy(m.master, host_blob, m.count * 4, hipMemcpyHostToDevice));
  REVO_HIP_TRY(hipMalloc(&m.ops, m.count * esize(p)));
  m.bytes = m.count * (4 + esize(p));
  int rc = launch_convert(base_prec(p), m.master, m.ops, (long long)m.count, s);
  if (rc) return rc;
  if (p == P_FP8) {
    REVO_HIP_TRY(hipMalloc(&m.ops8, m.count));
    REVO_HIP_TRY(hipMalloc(&m.wscale, m.count / 64 * 4));  // >= rows of all matrices (cols >= 192)
    m.nact = 4 * (ne + nd) + 1;
    REVO_HIP_TRY(hipMalloc(&m.act_scale, m.nact * 4));
    REVO_HIP_TRY(hipMalloc(&m.act_absmax, m.nact * 4));
    m.nattn = 3 * (m.He * ne + m.Hd * nd);
    REVO_HIP_TRY(hipMalloc(&m.attn_absmax, m.nattn * 4));
    REVO_HIP_TRY(hipMalloc(&m.attn_exp, m.nattn * 4));
    REVO_HIP_TRY(hipMalloc(&m.attn_inv, m.nattn * 4));
    m.bytes += m.count + m.count / 64 * 4 + m.nact * 8 + m.nattn * 12;
    if ((rc = model_reset_calibration(m, s))) return rc;
  }
  REVO_HIP_TRY(hipStreamSynchronize(s));

  size_t pos = 0, srow = 0;
  auto mat = [&](size_t rows, size_t cols) {
    const void* q = (const char*)m.ops + pos * esize(p);
    pos += rows * cols;
    return q;
  };
  // FP8 copy of the matrix just taken by mat() with its row scales
  auto mat8 = [&](size_t rows, size_t cols, const uint8_t** w8, const float** sc) -> int {
    if (p != P_FP8) return 0;
    const size_t off = pos - rows * cols;
    *w8 = m.ops8 + off;
    *sc = m.wscale + srow;
    const int e = launch_quantize_rows(m.master + off, (int)rows, (int)cols, m.ops8 + off, m.wscale + srow, s);
    srow += rows;
    return e;
  };
  auto vec = [&](size_t len) {
    const float* q = m.master + pos;
    pos += len;
    return q;
  };
  auto block = [&](int D) {
    BlockW b;
    b.ln1_g = vec(D); b.ln1_b = vec(D);
    b.qkv_w = mat(3 * D, D); rc |= mat8(3 * D, D, &b.qkv_w8, &b.qkv_s); b.qkv_b = vec(3 * D);
    b.proj_w = mat(D, D); rc |= mat8(D, D, &b.proj_w8, &b.proj_s); b.proj_b = vec(D);
    b.ln2_g = vec(D); b.ln2_b = vec(D);
    b.fc1_w = mat(4 * D, D); rc |= mat8(4 * D, D, &b.fc1_w8, &b.fc1_s); b.fc1_b = vec(4 * D);
    b.fc2_w = mat(D, 4 * D); rc |= mat8(D, 4 * D, &b.fc2_w8, &b.fc2_s); b.fc2_b = vec(D);
    return b;
  };
  const int L = m.tub_len();
  m.emb_w = mat(m.De, L); m.emb_b = vec(m.De);
  m.enc.clear();
  for (int i = 0; i < ne; ++i) m.enc.push_back(block(m.De));
  m.enc_g = vec(m.De); m.enc_b = vec(m.De);
  m.e2d_w = mat(m.Dd, m.De); rc |= mat8(m.Dd, m.De, &m.e2d_w8, &m.e2d_s); m.e2d_b = vec(m.Dd);
  m.dec.clear();
  for (int i = 0; i < nd; ++i) m.dec.push_back(block(m.Dd));
  m.dec_g = vec(m.Dd); m.dec_b = vec(m.Dd);
  m.head_w = mat(L, m.Dd); m.head_b = vec(L);
  if (rc) return -5;
  if (p == P_FP8) REVO_HIP_TRY(hipStreamSynchronize(s));
  return pos == m.count ? 0 : -22;
}

int model_reset_calibration(ModelW& m, hipStream_t s) {
  if (m.prec != P_FP8) return -22;
  int rc = launch_fill_zero(m.act_absmax, m.nact * 4, s);
  if (!rc) rc = launch_fill_zero(m.attn_absmax, m.nattn * 4, s);
  if (rc) return rc;
  m.calibrated = false;
  rc = launch_scales_from_absmax(m.act_absmax, m.act_scale, m.nact, s);
  return rc ? rc : launch_attn_scales(m.attn_absmax, m.attn_exp, m.attn_inv, m.nattn, s);
}

int model_finish_calibration(ModelW& m, hipStream_t s) {
  if (m.prec != P_FP8) return -22;
  int rc = launch_scales_from_absmax(m.act_absmax, m.act_scale, m.nact, s);
  if (!rc) rc = launch_attn_scales(m.attn_absmax, m.attn_exp, m.attn_inv, m.nattn, s);
  if (rc) return rc;
  REVO_HIP_TRY(hipStreamSynchronize(s));
  m.calibrated = true;
  return 0;
}

void model_free(ModelW& m) {
  void* p[] = {m.master, m.ops, m.ops8, m.wscale, m.act_scale, m.act_absmax, m.attn_absmax, m.attn_exp, m.attn_inv};
  for (void* q : p)
    if (q) (void)hipFree(q);
  m.master = nullptr; m.ops = nullptr; m.ops8 = nullptr; m.wscale = nullptr;
  m.act_scale = nullptr; m.act_absmax = nullptr;
  m.attn_absmax = nullptr; m.attn_exp = nullptr; m.attn_inv = nullptr;
}

int prof_init(Prof& p, int events) {
  p.pool.resize(events);
  for (auto& e : p.pool) REVO_HIP_TRY(hipEventCreate(&e));
  p.on = true;
  return 0;
}

void prof_free(Prof& p) {
  for (auto& e : p.pool) (void)hipEventDestroy(e);
  p.pool.clear();
  p.on = false;
}

int prof_collect(Prof& p) {
  for (const auto& r : p.recs) {
    float ms = 0.0f;
    REVO_HIP_TRY(hipEventElapsedTime(&ms, p.pool[r.a], p.pool[r.b]));
    p.ms[r.kind] += ms;
    p.flop[r.kind] += r.flop;
    p.count[r.kind] += 1;
  }
  p.recs.clear();
  p.used = 0;
  return 0;
}

namespace {

// Event pair around one launch when profiling; no-op otherwise.
struct ProfScope {
  Prof& p;
  hipStream_t s;
  int a = -1, kind;
  double flop;
  ProfScope(Prof& p_, hipStream_t s_, int kind_, double flop_) : p(p_), s(s_), kind(kind_), flop(flop_) {
    if (p.on && (!p.attn_only || kind == PK_ATTN || kind == PK_FORWARD) && p.used + 2 <= (int)p.pool.size()) {
      a = p.used;
      p.used += 2;
      (void)hipEventRecord(p.pool[a], s);
    }
  }
  ~ProfScope() {
    if (a >= 0) {
      (void)hipEventRecord(p.pool[a + 1], s);
      p.recs.push_back({a, a + 1, kind, flop});
    }
  }
};

}  // namespace

int request_tokens(int H, int W, int J) { return J * cdiv(H, REVO_PATCH) * cdiv(W, REVO_PATCH); }

size_t workspace_bytes(const ModelW& m, int cap, int max_req) {
  const size_t e = esize(m.prec);
  const size_t ld = (size_t)cap + 64;
  const size_t De = m.De;
  size_t b = 0;
  b += (size_t)cap * De * 4;             // h
  b += (size_t)cap * De * e;             // a
  b += 2 * (size_t)m.He * ld * 64 * e;   // q, k
  b += (size_t)m.He * 64 * ld * e;       // vt
  b += (size_t)cap * De * e;             // o
  b += (size_t)cap * 4 * De * e;         // hid
  b += (size_t)cap * m.Dd * 4;           // z
  b += (size_t)cap * m.Dd * e;           // ahead (target rows <= cap)
  b += (size_t)max_req * sizeof(ReqDesc) + 2 * (size_t)(cap / 128 + max_req + 1) * 4 + HDR_N * 4;
  return b + 16 * 256;
}

int workspace_alloc(Workspace& w, const ModelW& m, int cap, int max_req, hipStream_t s) {
  w.cap = cap; w.head_cap = cap; w.ld = cap + 64; w.max_req = max_req; w.prec = m.prec;
  w.max_work = cap / 128 + max_req + 1;
  const size_t e = esize(m.prec);
  const size_t De = m.De;
  auto get = [&](void** p, size_t bytes) -> int {
    REVO_HIP_TRY(hipMalloc(p, bytes));
    w.bytes += bytes;
    return launch_fill_zero(*p, (long long)bytes, s);
  };
  int rc = 0;
  rc |= get((void**)&w.h, (size_t)cap * De * 4);
  rc |= get(&w.a, (size_t)cap * De * e);
  rc |= get(&w.q, (size_t)m.He * w.ld * 64 * e);
  rc |= get(&w.k, (size_t)m.He * w.ld * 64 * e);
  rc |= get(&w.vt, (size_t)m.He * 64 * w.ld * e);
  rc |= get(&w.o, (size_t)cap * De * e);
  rc |= get(&w.hid, (size_t)cap * 4 * De * e);
  rc |= get((void**)&w.z, (size_t)cap * m.Dd * 4);
  rc |= get(&w.ahead, (size_t)cap * m.Dd * e);
  rc |= get((void**)&w.d_reqs, (size_t)max_req * sizeof(ReqDesc));
  rc |= get((void**)&w.d_work, 2 * (size_t)w.max_work * 4);  // all q-tiles, then target-tubelet q-tiles
  rc |= get((void**)&w.d_hdr, HDR_N * 4);
  if (rc) return rc < 0 ? rc : -5;
  for (int sl = 0; sl < WS_SLOTS; ++sl) {
    REVO_HIP_TRY(hipHostMalloc((void**)&w.h_reqs_slot[sl], (size_t)max_req * sizeof(ReqDesc), hipHostMallocDefault));
    REVO_HIP_TRY(hipHostMalloc((void**)&w.h_work_slot[sl], 2 * (size_t)w.max_work * 4, hipHostMallocDefault));
    REVO_HIP_TRY(hipHostMalloc((void**)&w.h_hdr_slot[sl], HDR_N * 4, hipHostMallocDefault));
    memset(w.h_reqs_slot[sl], 0, (size_t)max_req * sizeof(ReqDesc));
  }
  w.h_reqs = w.h_reqs_slot[0];
  REVO_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

void workspace_free(Workspace& w) {
  prof_free(w.prof);
  for (auto& g : w.graph)
    if (g) (void)hipGraphExecDestroy(g);
  void* dev[] = {w.h, w.a, w.q, w.k, w.vt, w.o, w.hid, w.z, w.ahead, w.d_reqs, w.d_work, w.d_hdr};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  for (int sl = 0; sl < WS_SLOTS; ++sl) {
    if (w.h_reqs_slot[sl]) (void)hipHostFree(w.h_reqs_slot[sl]);
    if (w.h_work_slot[sl]) (void)hipHostFree(w.h_work_slot[sl]);
    if (w.h_hdr_slot[sl]) (void)hipHostFree(w.h_hdr_slot[sl]);
  }
  w = Workspace();
}

namespace {

// Launch sequence of the network.  Grid sizes come from the arguments (exact
// counts when eager, bucket capacities when captured); with dyn set, the
// kernels read the live counts from the device batch header.
int enqueue_net(const ModelW& m, Workspace& w, int Mg, int Mhg, int nworkg, int nworkg_last, int nrec, int nall,
                int max_pix, int composite, bool dyn, double Mreal, double Mh_real, double attn_pairs,
                double attn_pairs_last, bool record, hipStream_t s) {
  const Prec pb = base_prec(m.prec);                       // embedding, attention, head, LN outputs
  const bool fp8 = m.prec == P_FP8 && m.calibrated && !record;  // FP8 block products
  const int* H = dyn ? w.d_hdr : nullptr;
  ProfScope whole(w.prof, s, PK_FORWARD, 0.0);
  auto gemm = [&](Prec p, int epi, int xm, const GemmArgs& ga, double rows) {
    ProfScope ps(w.prof, s, PK_GEMM, 2.0 * rows * ga.N * ga.K);
    return launch_gemm(p, epi, xm, ga, s);
  };
  auto ln = [&](const float* x, const float* gg, const float* bb, void* y, int rows, int D, const ReqDesc* rq,
                int nq, const int* dyn_rows) {
    ProfScope ps(w.prof, s, PK_OTHER, 0.0);
    return launch_layernorm(pb, x, gg, bb, y, rows, D, rq, nq, s, dyn_rows, H ? H + HDR_NREC : nullptr);
  };
  auto ln8 = [&](const float* x, const float* gg, const float* bb, int rows, int D, int act) {
    ProfScope ps(w.prof, s, PK_OTHER, 0.0);
    return launch_layernorm_fp8(x, gg, bb, (uint8_t*)w.a, m.act_scale + act, rows, D, s, H ? H + HDR_M : nullptr);
  };
  // calibration: raise the maxima of a BF16 activation that an FP8 product will take
  auto probe = [&](const void* x, int D, int act) {
    return record ? launch_absmax((const __bf16*)x, Mg, D, w.d_reqs, nrec, m.act_absmax + act, s) : 0;
  };
  int rc = 0;
  if (nrec > 0) {
    GemmArgs g;
    memset(&g, 0, sizeof(g));
    g.reqs = w.d_reqs; g.nreq = nrec; g.channels = m.C;
    g.dyn_m = H ? H + HDR_M : nullptr;
    g.dyn_nreq = H ? H + HDR_NREC : nullptr;
    // tubelet embedding + PE: the tubelet vectors are packed into the MLP
    // hidden buffer (free at this point) when they fit, then multiplied as a
    // dense operand; longer tubelets gather inside the product
    g.M = Mg; g.N = m.De; g.K = m.tub_len(); g.W = m.emb_w; g.bias = m.emb_b; g.out = w.h; g.ldo = m.De;
    if (m.tub_len() <= 4 * m.De) {
      {
        ProfScope ps(w.prof, s, PK_OTHER, 0.0);
        if ((rc = launch_tubelet_pack(pb, g, w.hid, s))) return rc;
      }
      GemmArgs ge = g;
      ge.X = w.hid;
      if ((rc = gemm(pb, EPI_PE, X_DENSE, ge, Mreal))) return rc;
    } else if ((rc = gemm(pb, EPI_PE, X_GATHER, g, Mreal))) {
      return rc;
    }

    AttnArgs at;
    memset(&at, 0, sizeof(at));
    at.q = w.q; at.k = w.k; at.vt = w.vt; at.o = w.o; at.ldqk = w.ld; at.ldv = w.ld;
    at.reqs = w.d_reqs; at.nreq = nrec; at.work = w.d_work; at.nwork = nworkg;
    at.dyn_nwork = H ? H + HDR_NWORK : nullptr;
    at.dyn_nreq = H ? H + HDR_NREC : nullptr;

    auto run_block = [&](const BlockW& b, float* x, int D, int heads, bool dec, int bi) -> int {
      int e;
      const int sq = m.act_slot(dec, bi, ACT_QKV), sp = m.act_slot(dec, bi, ACT_PROJ);
      const int s1 = m.act_slot(dec, bi, ACT_FC1), s2 = m.act_slot(dec, bi, ACT_FC2);
      const Prec pg = fp8 ? P_FP8 : pb;
      if ((e = fp8 ? ln8(x, b.ln1_g, b.ln1_b, Mg, D, sq) : ln(x, b.ln1_g, b.ln1_b, w.a, Mg, D, nullptr, 0, H ? H + HDR_M : nullptr))) return e;
      if ((e = probe(w.a, D, sq))) return e;
      GemmArgs q = g;
      q.X = w.a; q.K = D; q.N = 3 * D; q.W = fp8 ? (const void*)b.qkv_w8 : b.qkv_w; q.bias = b.qkv_b;
      q.q = w.q; q.k = w.k; q.vt = w.vt; q.heads = heads; q.ldqk = w.ld; q.ldv = w.ld;
      q.qscale = 1.4426950408889634f / 8.0f;  // log2(e) / sqrt(64)
      const int ao = m.attn_off(dec, bi);
      // FP8: E4M3 Q / K / V^T with per-head power-of-two scales for the FP8 attention
      if (fp8) { q.wscale = b.qkv_s; q.xscale = m.act_scale + sq; q.head_inv = m.attn_inv + ao; }
      if ((e = gemm(pg, EPI_QKV, X_DENSE, q, Mreal))) return e;
      if (record && (e = launch_attn_absmax((const __bf16*)w.q, (const __bf16*)w.k, (const __bf16*)w.vt, heads, w.ld, Mg,
                                            w.d_reqs, nrec, m.attn_absmax + ao, s)))
        return e;
      // the last decoder block only needs the queries of the target tubelet:
      // its other tokens feed nothing after it (the head reads the target rows)
      const bool last = dec && bi == m.nd - 1;
      AttnArgs ab = at;
      ab.heads = heads;
      ab.o_scale = fp8 ? m.act_scale + sp : nullptr;
      ab.qkv_exp = fp8 ? m.attn_exp + ao : nullptr;
      if (last) {
        ab.work = w.d_work + w.max_work;
        ab.nwork = nworkg_last;
        ab.dyn_nwork = H ? H + HDR_NWORK_LAST : nullptr;
      }
      {
        ProfScope ps(w.prof, s, PK_ATTN, 4.0 * 64.0 * heads * (last ? attn_pairs_last : attn_pairs));
        if ((e = launch_attention(fp8 ? P_FP8 : pb, ab, s))) return e;
      }
      if ((e = probe(w.o, D, sp))) return e;
      GemmArgs pr = g;
      pr.X = w.o; pr.K = D; pr.N = D; pr.W = fp8 ? (const void*)b.proj_w8 : b.proj_w; pr.bias = b.proj_b;
      pr.out = x; pr.ldo = D;
      if (fp8) { pr.wscale = b.proj_s; pr.xscale = m.act_scale + sp; }
      if ((e = gemm(pg, EPI_RESIDUAL, X_DENSE, pr, Mreal))) return e;
      if ((e = fp8 ? ln8(x, b.ln2_g, b.ln2_b, Mg, D, s1) : ln(x, b.ln2_g, b.ln2_b, w.a, Mg, D, nullptr, 0, H ? H + HDR_M : nullptr))) return e;
      if ((e = probe(w.a, D, s1))) return e;
      GemmArgs f1 = g;
      f1.X = w.a; f1.K = D; f1.N = 4 * D; f1.W = fp8 ? (const void*)b.fc1_w8 : b.fc1_w; f1.bias = b.fc1_b;
      f1.out = w.hid; f1.ldo = 4 * D;
      if (fp8) { f1.wscale = b.fc1_s; f1.xscale = m.act_scale + s1; f1.out_scale = m.act_scale + s2; }
      if ((e = gemm(pg, EPI_GELU, X_DENSE, f1, Mreal))) return e;
      if ((e = probe(w.hid, 4 * D, s2))) return e;
      GemmArgs f2 = g;
      f2.X = w.hid; f2.K = 4 * D; f2.N = D; f2.W = fp8 ? (const void*)b.fc2_w8 : b.fc2_w; f2.bias = b.fc2_b;
      f2.out = x; f2.ldo = D;
      if (fp8) { f2.wscale = b.fc2_s; f2.xscale = m.act_scale + s2; }
      return gemm(pg, EPI_RESIDUAL, X_DENSE, f2, Mreal);
    };
    for (int i = 0; i < m.ne; ++i)
      if ((rc = run_block(m.enc[i], w.h, m.De, m.He, false, i))) return rc;
    // encoder norm, projection to the decoder width + PE
    const int se = m.act_e2d();
    if ((rc = fp8 ? ln8(w.h, m.enc_g, m.enc_b, Mg, m.De, se)
                  : ln(w.h, m.enc_g, m.enc_b, w.a, Mg, m.De, nullptr, 0, H ? H + HDR_M : nullptr))) return rc;
    if ((rc = probe(w.a, m.De, se))) return rc;
    GemmArgs e2 = g;
    e2.X = w.a; e2.K = m.De; e2.N = m.Dd; e2.W = fp8 ? (const void*)m.e2d_w8 : m.e2d_w; e2.bias = m.e2d_b;
    e2.out = w.z; e2.ldo = m.Dd;
    if (fp8) { e2.wscale = m.e2d_s; e2.xscale = m.act_scale + se; }
    if ((rc = gemm(fp8 ? P_FP8 : pb, EPI_PE, X_DENSE, e2, Mreal))) return rc;
    for (int i = 0; i < m.nd; ++i)
      if ((rc = run_block(m.dec[i], w.z, m.Dd, m.Hd, true, i))) return rc;
    // decoder norm and head on the target tubelet only, target time slot only
    if ((rc = ln(w.z, m.dec_g, m.dec_b, w.ahead, Mhg, m.Dd, w.d_reqs, nrec, H ? H + HDR_MH : nullptr))) return rc;
    const int slot = (m.T - 1) * 256 * m.C;
    GemmArgs hd = g;
    hd.M = Mhg; hd.X = w.ahead; hd.K = m.Dd; hd.N = 256 * m.C;
    hd.dyn_m = H ? H + HDR_MH : nullptr;
    hd.W = (const char*)m.head_w + (size_t)slot * m.Dd * esize(m.prec);
    hd.bias = m.head_b + slot;
    if ((rc = gemm(pb, EPI_HEAD, X_DENSE, hd, Mh_real))) return rc;
  }
  ProfScope ps(w.prof, s, PK_OTHER, 0.0);
  return launch_composite(w.d_reqs, nall, m.C, max_pix, composite, s, H ? H + HDR_NALL : nullptr);
}

}  // namespace

int forward(const ModelW& m, Workspace& w, int slot, int nrec, int nall, int composite, bool use_graph,
            hipStream_t s, bool record) {
  if (nall <= 0) return 0;
  if (nall > w.max_req || nrec > nall || slot < 0 || slot >= WS_SLOTS) return -22;
  ReqDesc* reqs = w.h_reqs_slot[slot];
  int* work = w.h_work_slot[slot];
  int* hdr = w.h_hdr_slot[slot];
  // token and head-row offsets, attention work list
  int M = 0, Mh = 0, nwork = 0, max_pix = 0;
  double Mreal = 0.0, attn_pairs = 0.0, attn_pairs_last = 0.0;
  int nwork_last = 0;
  int* work_last = work + w.max_work;
  for (int r = 0; r < nall; ++r) {
    ReqDesc& d = reqs[r];
    d.gy = cdiv(d.H, REVO_PATCH);
    d.gx = cdiv(d.W, REVO_PATCH);
    d.P = d.gy * d.gx;
    if (d.H * d.W > max_pix) max_pix = d.H * d.W;
    if (r >= nrec) { d.tok_off = M; d.head_off = Mh; continue; }
    // every request starts a V^T key group (16 keys for BF16, 64 for FP8
    // attention) with 16-byte aligned columns
    const int al = token_align(m.prec);
    M = (M + al - 1) / al * al;
    d.tok_off = M;
    d.head_off = Mh;
    const int N = d.J * d.P;
    for (int qt = 0; qt * 128 < N; ++qt) {
      if (nwork >= w.max_work) return -22;
      work[nwork++] = (r << 16) | qt;
    }
    for (int qt = 0; qt * 128 < d.P; ++qt) {
      if (nwork_last >= w.max_work) return -22;
      work_last[nwork_last++] = (r << 16) | ATTN_TARGET_TILE | qt;
    }
    M += N;
    Mh += d.P;
    Mreal += N;
    attn_pairs += (double)N * N;
    attn_pairs_last += (double)N * d.P;
  }
  if (M > w.cap) return -22;
  hdr[HDR_M] = M; hdr[HDR_MH] = Mh; hdr[HDR_NREC] = nrec; hdr[HDR_NALL] = nall; hdr[HDR_NWORK] = nwork;
  hdr[HDR_NWORK_LAST] = nwork_last;
  REVO_HIP_TRY(hipMemcpyAsync(w.d_reqs, reqs, (size_t)nall * sizeof(ReqDesc), hipMemcpyHostToDevice, s));
  REVO_HIP_TRY(hipMemcpyAsync(w.d_hdr, hdr, HDR_N * 4, hipMemcpyHostToDevice, s));
  if (nwork > 0) REVO_HIP_TRY(hipMemcpyAsync(w.d_work, work, (size_t)nwork * 4, hipMemcpyHostToDevice, s));
  if (nwork_last > 0)
    REVO_HIP_TRY(hipMemcpyAsync(w.d_work + w.max_work, work_last, (size_t)nwork_last * 4, hipMemcpyHostToDevice, s));

  if (!use_graph || w.prof.on || record) {
    return enqueue_net(m, w, M, Mh, nwork, nwork_last, nrec, nall, max_pix, composite, false, Mreal, Mh, attn_pairs,
                       attn_pairs_last, record, s);
  }
  // smallest capacity bucket holding this batch; capture its graph once
  int b = 0;
  while (b + 1 < WS_BUCKETS && (w.cap >> (WS_BUCKETS - 1 - b)) < M) ++b;
  const int capM = w.cap >> (WS_BUCKETS - 1 - b);
  if (!w.graph[b]) {
    const int capW = capM / 128 + w.max_req;
    const int capPix = 4096 * 4096;
    hipGraph_t g = nullptr;
    REVO_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int capWn = capW < w.max_work ? capW : w.max_work;
    int rc = enqueue_net(m, w, capM, capM, capWn, capWn, w.max_req, w.max_req, capPix, composite, true, 0.0, 0.0, 0.0,
                         0.0, false, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return -5;
    e = hipGraphInstantiate(&w.graph[b], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { w.graph[b] = nullptr; return -5; }
  }
  REVO_HIP_TRY(hipGraphLaunch(w.graph[b], s));
  return 0;
}

}  // namespace revo
