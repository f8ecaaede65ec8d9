// trs_host.cpp -- host runtime of libtrs: context, rule compiler, term
// loader, round driver and read-back behind the C-ABI of include/trs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "trs.h"
#include "trs_kernels.h"
#include "trs_layout.h"
#include "trs_mlp.h"

namespace {

const char *kStatusText[] = {"ok",         "bad argument", "call out of order", "invalid rule",
                             "invalid term", "node pool exhausted", "round limit reached",
                             "HIP runtime error", "compiled-table limit exceeded",
                             "internal error"};

}  // namespace

// A launch shape chosen by the autotuner and its device time.
struct Tuned {
  int block, npt, grid;
  double ms;
};

struct trs_ctx {
  trs_config cfg{};
  int A = 0;
  std::string err;

  // rewrite system
  bool rules_loaded = false;
  int n_sym = 0, n_rules = 0;
  std::vector<int32_t> arity;
  std::vector<uint8_t> has_rules;
  std::vector<int32_t> tab;

  // input terms (host image of the initial pool, slots 0 .. n_init-1)
  bool terms_loaded = false;
  int n_terms = 0;
  std::vector<int32_t> roots;
  int64_t n_init = 0;
  std::vector<int32_t> img_hss, img_args, img_rc, img_par;
  std::vector<uint8_t> img_state;
  bool img_on_device = false;  // pristine copy uploaded since the last load_terms

  // device side
  bool dev_ready = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Pool pool{};
  Ctl *d_ctl = nullptr;
  Ctl *h_ctl = nullptr;  // pinned
  // pristine device copy of the initial pool image (restored D2D by every
  // normalisation, so repeated runs need no host transfer)
  int32_t *d_img_hss = nullptr, *d_img_args = nullptr, *d_img_rc = nullptr;
  int32_t *d_img_par = nullptr;
  uint8_t *d_img_state = nullptr;
  int32_t stamp_base = 1;  // notification stamps of the next run start here
  int32_t *d_tab = nullptr;
  unsigned long long *d_bar = nullptr;
  std::vector<void *> owned;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int cu_count = 0;
  unsigned long long *h_zero = nullptr;  // pinned zero for barrier resets
  // captured chunk of rounds (one launch per round)
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int g_grid = 0, g_block = 0, g_k = 0, g_sgrid = 0;
  size_t g_lds = 0;
  RoundArgs g_args;  // kernel arguments baked into the captured chunk

  // frontier predictor (learned mode) and tracing
  std::vector<uint16_t> pred;  // installed parameters (empty: none)
  bool pred_dirty = false;
  uint16_t *d_pred = nullptr;
  int32_t *d_arity = nullptr;
  float *d_pprobs = nullptr, *d_ploss = nullptr;
  uint64_t *d_prec = nullptr;
  unsigned long long *d_trace_rec = nullptr;
  int32_t *d_trace_n = nullptr;
  int64_t trace_alloc = 0, trace_count = 0;
  // autotuner results for the loaded terms, per mode: block, npt, ms
  std::map<int, Tuned> tuned;  // autotuned launch shape per mode

  // results of the last normalisation
  bool normalized = false;
  int64_t n_final = 0;
  int64_t fs_final[2] = {0, 0};  // free-stack sizes at the end of the run
  std::vector<int64_t> rule_counts;
  bool cache_valid = false;
  std::vector<int32_t> c_hss, c_args;
  std::vector<uint8_t> c_state;

  trs_status fail(trs_status s, const std::string &msg) {
    err = msg;
    return s;
  }
};

namespace {

// ------------------------------------------------------------------ parsing

// length of the prefix code starting at code[p] (variables, coded < 0, are
// leaves); -1 if it runs past end or names an unknown symbol
int64_t prefix_len(const std::vector<int32_t> &arity, const int32_t *code, int64_t p,
                   int64_t end) {
  int64_t need = 1, q = p;
  while (need > 0) {
    if (q >= end) return -1;
    int32_t c = code[q++];
    need--;
    if (c >= 0) {
      if (c >= (int32_t)arity.size()) return -1;
      need += arity[c];
    }
  }
  return q - p;
}

struct PNode {
  int parent = -1, pos = 0, sym = -1, var = -1;
  std::string key;
};

struct RNode {
  int sym = -1, var = -1;
  std::vector<int> kids;
};

std::string sym_key(int sym) { return "s" + std::to_string(sym); }
std::string var_key(int var) { return "v" + std::to_string(var); }

// build the pattern tree of a left-hand side given in prefix code
bool parse_lhs(const std::vector<int32_t> &arity, const int32_t *c, int64_t len,
               std::vector<PNode> &out) {
  out.clear();
  struct Fr {
    int node, next, ar;
  };
  std::vector<Fr> st;
  for (int64_t i = 0; i < len; i++) {
    PNode pn;
    if (!st.empty()) {
      pn.parent = st.back().node;
      pn.pos = st.back().next++;
    }
    if (c[i] < 0) {
      pn.var = -1 - c[i];
    } else {
      pn.sym = c[i];
    }
    out.push_back(pn);
    int me = (int)out.size() - 1;
    if (c[i] >= 0 && arity[c[i]] > 0) st.push_back({me, 0, arity[c[i]]});
    while (!st.empty() && st.back().next == st.back().ar) st.pop_back();
  }
  // canonical keys, children first (prefix order reversed)
  std::vector<std::vector<int>> kids(out.size());
  for (size_t k = 1; k < out.size(); k++) kids[out[k].parent].push_back((int)k);
  for (int k = (int)out.size() - 1; k >= 0; k--) {
    if (out[k].var >= 0) {
      out[k].key = var_key(out[k].var);
    } else {
      std::string s = sym_key(out[k].sym) + "(";
      for (size_t j = 0; j < kids[k].size(); j++) {
        if (j) s += ",";
        s += out[kids[k][j]].key;
      }
      out[k].key = s + ")";
    }
  }
  return true;
}

void parse_rhs(const std::vector<int32_t> &arity, const int32_t *c, int64_t len,
               std::vector<RNode> &out) {
  out.clear();
  struct Fr {
    int node, ar;
  };
  std::vector<Fr> st;
  for (int64_t i = 0; i < len; i++) {
    RNode rn;
    if (c[i] < 0)
      rn.var = -1 - c[i];
    else
      rn.sym = c[i];
    out.push_back(rn);
    int me = (int)out.size() - 1;
    if (!st.empty()) out[st.back().node].kids.push_back(me);
    if (c[i] >= 0 && arity[c[i]] > 0) st.push_back({me, arity[c[i]]});
    while (!st.empty() && (int)out[st.back().node].kids.size() == st.back().ar) st.pop_back();
  }
}

std::string rhs_key(const std::vector<RNode> &R, int k) {
  if (R[k].var >= 0) return var_key(R[k].var);
  std::string s = sym_key(R[k].sym) + "(";
  for (size_t j = 0; j < R[k].kids.size(); j++) {
    if (j) s += ",";
    s += rhs_key(R, R[k].kids[j]);
  }
  return s + ")";
}

struct Program {
  std::vector<int32_t> words;  // program with offsets relative to its start
};

// Compile one rule into its table program.  Returns TRS_OK or an error with
// a message in *msg.
trs_status compile_rule(int rid, const std::vector<int32_t> &arity,
                        const std::vector<uint8_t> &has_rules, const std::vector<PNode> &P,
                        const std::vector<RNode> &R, Program &prog, std::string *msg) {
  const int npat = (int)P.size() - 1;
  if (npat > TRS_MAX_PATTERN) {
    *msg = "rule " + std::to_string(rid) + ": left-hand side too large";
    return TRS_E_LIMIT;
  }
  std::map<int, int> var_node;  // variable -> pattern node
  std::map<std::string, int> lhs_sub;  // non-variable subterm key -> pattern node (k >= 1)
  for (int k = 1; k <= npat; k++) {
    if (P[k].var >= 0)
      var_node[P[k].var] = k;
    else if (!lhs_sub.count(P[k].key))
      lhs_sub[P[k].key] = k;
  }
  struct NewNode {
    int sym, rc;
    bool nf;
    std::vector<int> ops;
  };
  std::vector<NewNode> nn;
  std::map<std::string, int> new_of;
  std::vector<int> refs(npat + 1, 0);
  // operand for RHS node k (not the root)
  std::function<int(int)> operand = [&](int k) -> int {
    if (R[k].var >= 0) {
      int pnode = var_node.at(R[k].var);
      refs[pnode]++;
      return pnode;
    }
    std::string key = rhs_key(R, k);
    auto it = lhs_sub.find(key);
    if (it != lhs_sub.end()) {  // reuse the matched node of an equal lhs subterm
      refs[it->second]++;
      return it->second;
    }
    auto jt = new_of.find(key);
    if (jt != new_of.end()) {  // equal subterms of one right-hand side are shared
      nn[jt->second].rc++;
      return -1 - jt->second;
    }
    NewNode x;
    x.sym = R[k].sym;
    x.rc = 1;
    for (int ch : R[k].kids) x.ops.push_back(operand(ch));
    bool nf = !has_rules[x.sym];
    for (int o : x.ops) nf = nf && (o >= 1 || nn[-1 - o].nf);
    x.nf = nf;
    nn.push_back(x);
    new_of[key] = (int)nn.size() - 1;
    return -1 - ((int)nn.size() - 1);
  };
  bool var_root = R[0].var >= 0;
  int rootpat = 0, rsym = -1;
  std::vector<int> rops;
  bool root_nf = false;
  if (var_root) {
    rootpat = var_node.at(R[0].var);
    root_nf = true;
  } else {
    rsym = R[0].sym;
    for (int ch : R[0].kids) rops.push_back(operand(ch));
    root_nf = !has_rules[rsym];
    for (int o : rops) root_nf = root_nf && (o >= 1 || nn[-1 - o].nf);
  }
  if ((int)nn.size() > TRS_MAX_NEW) {
    *msg = "rule " + std::to_string(rid) + ": right-hand side creates too many nodes";
    return TRS_E_LIMIT;
  }
  // parent hint of each new node: the first node that references it (the
  // root, coded 0, or new node j, coded j+1)
  std::vector<int> referrer(nn.size(), -1);
  for (int o : rops)
    if (o < 0 && referrer[-1 - o] < 0) referrer[-1 - o] = 0;
  for (size_t j = 0; j < nn.size(); j++)
    for (int o : nn[j].ops)
      if (o < 0 && referrer[-1 - o] < 0) referrer[-1 - o] = (int)j + 1;
  // a node is ready at birth when all its arguments are normal forms at birth
  auto ready_ops = [&](const std::vector<int> &ops) {
    for (int o : ops)
      if (!(o >= 1 || nn[-1 - o].nf)) return false;
    return true;
  };
  const bool root_ready = !var_root && !root_nf && ready_ops(rops);
  for (auto &x : nn)
    if (x.rc > 63) {
      *msg = "rule " + std::to_string(rid) + ": a right-hand-side node is shared too often";
      return TRS_E_LIMIT;
    }
  std::vector<std::pair<int, int>> pos, neg;
  for (int k = 1; k <= npat; k++) {
    int d = refs[k] - (P[k].parent == 0 ? 1 : 0);
    if (d > 0) pos.push_back({k, d});
    if (d < 0) neg.push_back({k, d});
  }
  std::vector<int32_t> &w = prog.words;
  w.assign(6, 0);
  w[0] = npat | ((int)nn.size() << 4) | ((int)var_root << 8) | ((int)root_nf << 9) |
         ((int)root_ready << 10) | ((int)pos.size() << 12) | ((int)neg.size() << 16) |
         (rootpat << 20);
  w[1] = rsym;
  w[5] = rid;
  for (int k = 1; k <= npat; k++) {
    int isvar = P[k].var >= 0;
    w.push_back(P[k].parent | (P[k].pos << 4) | (isvar << 8) | ((isvar ? 0 : P[k].sym) << 16));
  }
  w[2] = (int32_t)w.size();
  for (int o : rops) w.push_back(o);
  w[3] = (int32_t)w.size();
  for (size_t j = 0; j < nn.size(); j++) {
    const auto &x = nn[j];
    const int rdy = !x.nf && ready_ops(x.ops);
    w.push_back(x.sym | (x.rc << 16) | ((int)x.nf << 22) | (rdy << 23) |
                (std::max(referrer[j], 0) << 24));
    for (int o : x.ops) w.push_back(o);
  }
  w[4] = (int32_t)w.size();
  for (auto &pr : pos) w.push_back(pr.first | ((pr.second & 0xff) << 8));
  for (auto &pr : neg) w.push_back(pr.first | ((pr.second & 0xff) << 8));
  return TRS_OK;
}

// defaults of trs_opts.nf_walk, nf_walk_wide and cont_passes (frontier
// modes): constructors one walk marks per round in rounds one workgroup runs
// and in wider rounds, and further same-round passes in rounds one
// workgroup runs (wider rounds run none unless cont_passes_wide asks)
#define TRS_DEFAULT_WALK 256
#define TRS_DEFAULT_WALK_WIDE 1
#define TRS_DEFAULT_CONT 64

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return (ctx)->fail(TRS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// two wake bits per slot, in 32-bit words, over the slots a sweep may read
size_t wake_bytes(int64_t N) { return (size_t)((N + (1 << 16)) / 16 + 1) * 4; }

struct Piece {
  void **dst;
  size_t bytes;
};

// device arrays of a context, in carving order
std::vector<Piece> device_pieces(trs_ctx *c, int64_t N, int A) {
  const size_t state_pad = 1 << 16;  // vector loads of the last tile stay in bounds
  return {
      {(void **)&c->pool.hss, (size_t)N * 4},
      {(void **)&c->pool.args, (size_t)N * A * 4},
      {(void **)&c->pool.state, (size_t)N + state_pad},
      {(void **)&c->pool.rc, (size_t)N * 4},
      {(void **)&c->pool.fstack0, (size_t)N * 4},
      {(void **)&c->pool.fstack1, (size_t)N * 4},
      {(void **)&c->pool.dead0, (size_t)N * 4},
      {(void **)&c->pool.dead1, (size_t)N * 4},
      {(void **)&c->d_ctl, sizeof(Ctl)},
      {(void **)&c->d_tab, (size_t)(TAB_MAX_WORDS + TAB_GATE_MAX_WORDS) * 4},
      {(void **)&c->d_bar, 256},
      {(void **)&c->d_img_hss, (size_t)N * 4},
      {(void **)&c->d_img_args, (size_t)N * A * 4},
      {(void **)&c->d_img_rc, (size_t)N * 4},
      {(void **)&c->d_img_state, (size_t)N},
      {(void **)&c->d_img_par, (size_t)N * 4},
      {(void **)&c->pool.par, (size_t)N * 4},
      {(void **)&c->pool.front0, (size_t)N * 4},
      {(void **)&c->pool.front1, (size_t)N * 4},
      {(void **)&c->pool.ret0, (size_t)N * 4},
      {(void **)&c->pool.ret1, (size_t)N * 4},
      {(void **)&c->pool.qstamp, (size_t)N * 4},
      {(void **)&c->pool.wake, wake_bytes(N)},
  };
}

size_t carve_bytes(const std::vector<Piece> &pieces) {
  size_t off = 0;
  for (auto &pc : pieces) {
    off = (off + 255) & ~(size_t)255;
    off += pc.bytes;
  }
  return off;
}

trs_status device_init(trs_ctx *c) {
  if (c->dev_ready) return TRS_OK;
  HIPCHK(c, hipSetDevice(c->cfg.device));
  hipDeviceProp_t prop;
  HIPCHK(c, hipGetDeviceProperties(&prop, c->cfg.device));
  c->cu_count = prop.multiProcessorCount;
  if (c->cfg.hip_stream) {
    c->stream = (hipStream_t)c->cfg.hip_stream;
  } else {
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  const int64_t N = c->cfg.pool_slots;
  const int A = c->A;
  std::vector<Piece> pieces = device_pieces(c, N, A);
  if (c->cfg.dev_mem) {
    size_t off = 0;
    char *base = (char *)c->cfg.dev_mem;
    for (auto &pc : pieces) {
      off = (off + 255) & ~(size_t)255;
      *pc.dst = base + off;
      off += pc.bytes;
    }
    if (off > (size_t)c->cfg.dev_bytes)
      return c->fail(TRS_E_ARG, "dev_mem too small: need " + std::to_string(off) + " bytes");
  } else {
    for (auto &pc : pieces) {
      HIPCHK(c, hipMalloc(pc.dst, pc.bytes));
      c->owned.push_back(*pc.dst);
    }
  }
  c->pool.N = N;
  HIPCHK(c, hipMemsetAsync(c->pool.qstamp, 0, (size_t)N * 4, c->stream));
  c->stamp_base = 1;
  HIPCHK(c, hipHostMalloc((void **)&c->h_ctl, sizeof(Ctl), hipHostMallocDefault));
  HIPCHK(c, hipHostMalloc((void **)&c->h_zero, 64, hipHostMallocDefault));
  std::memset(c->h_zero, 0, 64);
  HIPCHK(c, hipEventCreate(&c->ev0));
  HIPCHK(c, hipEventCreate(&c->ev1));
  c->dev_ready = true;
  return TRS_OK;
}

int default_block() { return 256; }
int default_npt() { return 16; }

}  // namespace

// ======================================================================= ABI

extern "C" {

int64_t trs_device_bytes(int64_t pool_slots, int32_t maxarity) {
  if (pool_slots < 2 || pool_slots > (1ll << 30) || maxarity < 1 || maxarity > TRS_MAX_ARITY)
    return -1;
  trs_ctx tmp;
  return (int64_t)carve_bytes(device_pieces(&tmp, pool_slots, maxarity));
}

const char *trs_status_str(trs_status s) {
  int i = -s;
  if (i < 0 || i >= (int)(sizeof(kStatusText) / sizeof(kStatusText[0]))) return "unknown status";
  return kStatusText[i];
}

const char *trs_last_error(trs_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void trs_default_opts(trs_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->mode = TRS_MODE_PLAIN;
  o->block = 0;
  o->nodes_per_thread = 0;
  o->rounds_per_poll = 0;
  o->max_rounds = 0;
  o->threshold = 0.1f;
  o->persistent = 0;
  o->trace = 0;
  o->trace_cap = 0;
  o->label_horizon = 0;
  o->sweep_every = 0;
  o->max_grid = 0;
  o->pf_depth = 0;
  o->nf_walk = 0;
  o->cont_passes = 0;
  o->nf_walk_wide = 0;
  o->cont_passes_wide = 0;
  o->place_fresh = 0;
}

trs_status trs_create(trs_ctx **out, const trs_config *cfg) {
  if (!out || !cfg) return TRS_E_ARG;
  *out = nullptr;
  if (cfg->pool_slots < 2 || cfg->pool_slots > (1ll << 30)) return TRS_E_ARG;
  if (cfg->maxarity < 0 || cfg->maxarity > TRS_MAX_ARITY) return TRS_E_ARG;
  if (cfg->dev_mem && cfg->dev_bytes <= 0) return TRS_E_ARG;
  trs_ctx *c = new (std::nothrow) trs_ctx();
  if (!c) return TRS_E_INTERNAL;
  c->cfg = *cfg;
  *out = c;
  return TRS_OK;
}

void trs_destroy(trs_ctx *c) {
  if (!c) return;
  if (c->dev_ready) {
    (void)hipStreamSynchronize(c->stream);
    for (void *p : c->owned) (void)hipFree(p);
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    if (c->h_zero) (void)hipHostFree(c->h_zero);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

trs_status trs_load_rules(trs_ctx *c, int32_t n_sym, const int32_t *arity, int32_t n_rules,
                          const int32_t *rule_off, const int32_t *rule_code, int64_t code_len) {
  if (!c) return TRS_E_ARG;
  if (n_sym <= 0 || n_sym > TRS_MAX_SYMBOLS || !arity || n_rules < 0 ||
      n_rules > TRS_MAX_RULES || (n_rules > 0 && (!rule_off || !rule_code)) || code_len < 0)
    return c->fail(TRS_E_ARG, "bad sizes or null pointers");
  c->rules_loaded = c->terms_loaded = c->normalized = false;
  c->pred.clear();  // predictor parameters belong to a symbol set
  std::vector<int32_t> ar(arity, arity + n_sym);
  int maxar = 0;
  for (int i = 0; i < n_sym; i++) {
    if (ar[i] < 0)
      return c->fail(TRS_E_RULE, "symbol " + std::to_string(i) + " has an invalid arity");
    if (ar[i] > TRS_MAX_ARITY)
      return c->fail(TRS_E_LIMIT, "symbol " + std::to_string(i) + ": arity above " +
                                      std::to_string(TRS_MAX_ARITY) + " is not compiled");
    maxar = std::max(maxar, ar[i]);
  }
  int A = c->cfg.maxarity ? c->cfg.maxarity : std::max(1, maxar);
  if (maxar > A)
    return c->fail(TRS_E_RULE, "a symbol's arity exceeds maxarity " + std::to_string(A));
  if (A > TRS_MAX_ARITY) return c->fail(TRS_E_LIMIT, "maxarity above 5 is not compiled");

  std::vector<std::vector<PNode>> lhs(n_rules);
  std::vector<std::vector<RNode>> rhs(n_rules);
  std::vector<uint8_t> has(n_sym, 0);
  for (int r = 0; r < n_rules; r++) {
    const std::string rn = "rule " + std::to_string(r) + ": ";
    int64_t b = rule_off[r], e = rule_off[r + 1];
    if (b < 0 || e > code_len || e <= b) return c->fail(TRS_E_RULE, rn + "bad offsets");
    int64_t ll = prefix_len(ar, rule_code, b, e);
    if (ll < 0) return c->fail(TRS_E_RULE, rn + "malformed left-hand side");
    int64_t rl = prefix_len(ar, rule_code, b + ll, e);
    if (rl < 0 || b + ll + rl != e) return c->fail(TRS_E_RULE, rn + "malformed right-hand side");
    // Definition 1 (1): the left-hand side is not a variable
    if (rule_code[b] < 0) return c->fail(TRS_E_RULE, rn + "left-hand side is a variable");
    std::vector<uint8_t> seen(256, 0);
    for (int64_t i = b; i < b + ll; i++) {
      if (rule_code[i] < 0) {
        int v = -1 - rule_code[i];
        if (v >= 256) return c->fail(TRS_E_LIMIT, rn + "too many variables");
        // left-linearity: each variable at most once in the left-hand side
        if (seen[v]) return c->fail(TRS_E_RULE, rn + "left-hand side is not linear");
        seen[v] = 1;
      }
    }
    for (int64_t i = b + ll; i < e; i++) {
      if (rule_code[i] < 0) {
        int v = -1 - rule_code[i];
        // Definition 1 (2): Var(r) is a subset of Var(l)
        if (v >= 256 || !seen[v])
          return c->fail(TRS_E_RULE, rn + "right-hand side variable not in left-hand side");
      }
    }
    parse_lhs(ar, rule_code + b, ll, lhs[r]);
    parse_rhs(ar, rule_code + b + ll, rl, rhs[r]);
    has[rule_code[b]] = 1;
  }
  // per-symbol grouping in priority order
  std::vector<std::vector<int>> by_sym(n_sym);
  for (int r = 0; r < n_rules; r++) by_sym[lhs[r][0].sym].push_back(r);
  std::vector<int32_t> tab(TAB_SYM + n_sym + n_rules, 0);
  tab[0] = n_sym;
  tab[1] = n_rules;
  tab[2] = A;
  int first = 0;
  std::vector<int> order;  // rule ids in grouped order
  for (int f = 0; f < n_sym; f++) {
    if (by_sym[f].size() > 255)
      return c->fail(TRS_E_LIMIT, "more than 255 rules for one symbol");
    // argument positions whose own entries some rule of f reads: a pattern
    // deeper than the argument's symbol, or a right-hand side that is the
    // variable bound to the argument (the root takes over its entries)
    int deep = 0;
    for (int r : by_sym[f]) {
      for (const PNode &q : lhs[r])
        if (q.parent > 0 && lhs[r][q.parent].parent == 0) deep |= 1 << lhs[r][q.parent].pos;
      if (rhs[r][0].var >= 0)
        for (const PNode &q : lhs[r])
          if (q.var == rhs[r][0].var && q.parent == 0) deep |= 1 << q.pos;
    }
    tab[TAB_SYM + f] = tab_sym_word(ar[f], (int)by_sym[f].size(), first, deep);
    for (int r : by_sym[f]) order.push_back(r);
    first += (int)by_sym[f].size();
  }
  for (size_t i = 0; i < order.size(); i++) {
    int r = order[i];
    Program prog;
    std::string msg;
    trs_status st = compile_rule(r, ar, has, lhs[r], rhs[r], prog, &msg);
    if (st != TRS_OK) return c->fail(st, msg);
    int32_t base = (int32_t)tab.size();
    tab[TAB_SYM + n_sym + i] = base;
    for (size_t j = 0; j < prog.words.size(); j++) {
      int32_t w = prog.words[j];
      if (j >= 2 && j <= 4) w += base;  // section offsets become absolute
      tab.push_back(w);
    }
  }
  tab[3] = (int32_t)tab.size();
  if (tab.size() > TAB_MAX_WORDS) return c->fail(TRS_E_LIMIT, "compiled tables too large");
  c->n_sym = n_sym;
  c->n_rules = n_rules;
  c->arity = ar;
  c->has_rules = has;
  c->tab = tab;
  c->A = A;
  c->rule_counts.assign(n_rules, 0);
  c->rules_loaded = true;
  return TRS_OK;
}

trs_status trs_load_terms(trs_ctx *c, int32_t n_terms, const int64_t *term_off,
                          const int32_t *term_code, int64_t code_len) {
  if (!c) return TRS_E_ARG;
  if (!c->rules_loaded) return c->fail(TRS_E_STATE, "load rules first");
  if (n_terms < 0 || (n_terms > 0 && (!term_off || !term_code)) || code_len < 0)
    return c->fail(TRS_E_ARG, "bad sizes or null pointers");
  c->terms_loaded = c->normalized = c->cache_valid = false;
  if (n_terms > 0 && (term_off[0] < 0 || term_off[n_terms] > code_len))
    return c->fail(TRS_E_ARG, "term offsets out of range");
  int64_t M = 0;
  for (int t = 0; t < n_terms; t++) {
    int64_t b = term_off[t], e = term_off[t + 1];
    if (e <= b) return c->fail(TRS_E_TERM, "term " + std::to_string(t) + " is empty");
    for (int64_t i = b; i < e; i++)
      if (term_code[i] < 0 || term_code[i] >= c->n_sym)
        return c->fail(TRS_E_TERM, "term " + std::to_string(t) + " is not ground / bad symbol");
    if (prefix_len(c->arity, term_code, b, e) != e - b)
      return c->fail(TRS_E_TERM, "term " + std::to_string(t) + " is malformed");
    M += e - b;
  }
  if (M + 1 > c->cfg.pool_slots)
    return c->fail(TRS_E_POOL, "initial terms need " + std::to_string(M + 1) + " slots");
  const int A = c->A;
  c->n_init = M + 1;
  c->img_hss.assign(M + 1, 0);
  c->img_args.assign((size_t)(M + 1) * A, 0);
  c->img_rc.assign(M + 1, 0);
  c->img_state.assign(M + 1, ST_FREE);
  c->img_par.assign(M + 1, 0);
  c->roots.assign(n_terms, 0);
  int64_t slot = 1;
  std::vector<std::pair<int64_t, int>> st;  // (parent slot, next arg)
  for (int t = 0; t < n_terms; t++) {
    int64_t b = term_off[t], e = term_off[t + 1];
    int64_t first = slot;
    c->roots[t] = (int32_t)first;
    st.clear();
    for (int64_t i = b; i < e; i++) {
      int32_t s = term_code[i];
      int64_t me = slot++;
      c->img_hss[me] = s;
      c->img_rc[me] = 1;  // one parent, or the root-table entry
      if (!st.empty()) {
        c->img_args[(size_t)st.back().first * A + st.back().second] = (int32_t)me;
        c->img_par[me] = (int32_t)st.back().first;
        st.back().second++;
      }
      if (c->arity[s] > 0) st.push_back({me, 0});
      while (!st.empty() && st.back().second == c->arity[c->img_hss[st.back().first]]) st.pop_back();
    }
    // constructor-only subterms are normal forms from the start: a node whose
    // symbol has no rules and whose arguments are all normal forms
    for (int64_t me = slot - 1; me >= first; me--) {
      int32_t s = c->img_hss[me];
      bool nf = !c->has_rules[s];
      for (int j = 0; j < c->arity[s] && nf; j++)
        nf = c->img_state[c->img_args[(size_t)me * A + j]] == ST_NF;
      c->img_state[me] = nf ? (uint8_t)ST_NF : (uint8_t)ST_ACTIVE;
    }
  }
  c->n_terms = n_terms;
  c->terms_loaded = true;
  c->img_on_device = false;
  c->tuned.clear();
  return TRS_OK;
}

trs_status trs_normalize(trs_ctx *c, const trs_opts *opts_in, trs_stats *stats) {
  if (!c) return TRS_E_ARG;
  if (!c->terms_loaded) return c->fail(TRS_E_STATE, "load rules and terms first");
  trs_opts o;
  if (opts_in)
    o = *opts_in;
  else
    trs_default_opts(&o);
  if (o.mode != TRS_MODE_PLAIN && o.mode != TRS_MODE_FRONTIER && o.mode != TRS_MODE_LEARNED)
    return c->fail(TRS_E_ARG, "unknown mode");
  if (o.mode == TRS_MODE_LEARNED) {
    if (c->pred.empty()) return c->fail(TRS_E_STATE, "learned mode needs trs_set_predictor");
    if (!(o.threshold >= 0.f && o.threshold <= 1.f))
      return c->fail(TRS_E_ARG, "threshold must be in [0, 1]");
  }
  if (o.trace < 0 || o.trace > 65536) return c->fail(TRS_E_ARG, "trace rate must be 0..65536");
  if (o.max_grid < 0 || o.max_grid > (1 << 20))
    return c->fail(TRS_E_ARG, "max_grid must be 0..2^20");
  if (o.pf_depth < -1 || o.pf_depth > 4) return c->fail(TRS_E_ARG, "pf_depth must be -1..4");
  if (o.nf_walk < -1 || o.nf_walk > (1 << 26) || o.nf_walk_wide < -1 ||
      o.nf_walk_wide > (1 << 26))
    return c->fail(TRS_E_ARG, "nf_walk and nf_walk_wide must be -1..2^26");
  if (o.cont_passes < -1 || o.cont_passes > (1 << 20) || o.cont_passes_wide < -1 ||
      o.cont_passes_wide > (1 << 20))
    return c->fail(TRS_E_ARG, "cont_passes and cont_passes_wide must be -1..2^20");
  if (o.place_fresh < 0 || o.place_fresh > 100)
    return c->fail(TRS_E_ARG, "place_fresh must be 0..100");
  if (o.label_horizon < 0 || o.sweep_every < -1)
    return c->fail(TRS_E_ARG, "label_horizon must be >= 0, sweep_every >= -1");
  if (o.trace && o.mode != TRS_MODE_PLAIN)
    return c->fail(TRS_E_ARG, "traces are logged by plain-mode runs");
  const int64_t tcap = o.trace_cap ? o.trace_cap : ((int64_t)1 << 24);
  if (o.trace && (tcap <= 0 || tcap > INT32_MAX))
    return c->fail(TRS_E_ARG, "trace_cap must be 1..2^31-1");
  const int B = o.block ? o.block : default_block();
  const int npt = o.nodes_per_thread ? o.nodes_per_thread : default_npt();
  if (B < 64 || B > 1024 || (B & 63)) return c->fail(TRS_E_ARG, "block must be 64..1024, /64");
  if (!(npt == 1 || npt == 2 || npt == 4 || npt == 8 || npt == 16))
    return c->fail(TRS_E_ARG, "nodes_per_thread must be 1, 2, 4, 8 or 16");
  if (B * npt > 16384) return c->fail(TRS_E_ARG, "block * nodes_per_thread above 16384");
  if (o.max_rounds < 0 || o.rounds_per_poll < 0) return c->fail(TRS_E_ARG, "negative limits");
  trs_status st = device_init(c);
  if (st != TRS_OK) return st;
  c->normalized = false;
  c->cache_valid = false;
  const int A = c->A;
  const int64_t M1 = c->n_init;
  hipStream_t s = c->stream;
  if (!c->img_on_device) {
    HIPCHK(c, hipMemcpyAsync(c->d_img_hss, c->img_hss.data(), M1 * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_img_args, c->img_args.data(), M1 * A * 4,
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_img_rc, c->img_rc.data(), M1 * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_img_state, c->img_state.data(), M1, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_img_par, c->img_par.data(), M1 * 4, hipMemcpyHostToDevice, s));
    c->img_on_device = true;
  }
  HIPCHK(c, hipMemcpyAsync(c->pool.hss, c->d_img_hss, M1 * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->pool.args, c->d_img_args, M1 * A * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->pool.rc, c->d_img_rc, M1 * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->pool.state, c->d_img_state, M1, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->pool.par, c->d_img_par, M1 * 4, hipMemcpyDeviceToDevice, s));
  if (o.mode == TRS_MODE_PLAIN)
    HIPCHK(c, hipMemsetAsync(c->pool.wake, 0, wake_bytes(c->cfg.pool_slots), s));
  HIPCHK(c, hipMemcpyAsync(c->d_tab, c->tab.data(), c->tab.size() * 4, hipMemcpyHostToDevice, s));
  std::memset(c->h_ctl, 0, sizeof(Ctl));
  c->h_ctl->n[0] = (int32_t)M1;
  c->h_ctl->peak_n = (int32_t)M1;
  // notification stamps grow by the rounds of every run; restart them (and
  // clear the stamp array) well before they could wrap
  if (c->stamp_base > (1 << 30)) {
    HIPCHK(c, hipMemsetAsync(c->pool.qstamp, 0, (size_t)c->cfg.pool_slots * 4, s));
    c->stamp_base = 1;
  }
  c->h_ctl->stamp_base = c->stamp_base;
  {
    // round 0 is a full sweep; the launch that runs it needs one workgroup
    // per tile (one in all when a single tile covers the pool)
    const int64_t tiles = (M1 + (int64_t)B * npt - 1) / ((int64_t)B * npt);
    c->h_ctl->next_need = (int32_t)std::max<int64_t>(1, tiles);
    // the state of round 0 as the first launch reads it: done, r, need, n,
    // free-stack sizes, list lengths and flags (all zero but need and n)
    c->h_ctl->pub[2] = c->h_ctl->next_need;
    c->h_ctl->pub[3] = (int32_t)M1;
    c->h_ctl->pub[10] = c->stamp_base;
  }
  HIPCHK(c, hipMemcpyAsync(c->d_ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, s));
  unsigned long long zero = 0;
  HIPCHK(c, hipMemcpyAsync(c->d_bar, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));

  // learned mode and tracing: per-slot round of the last change (initial
  // nodes: round 0), trace buffer and the per-slot reference to the latest
  // record (all ones: none)
  const bool track = o.mode == TRS_MODE_LEARNED || o.trace;
  if (track && !c->pool.lastchg) {
    HIPCHK(c, hipMalloc(&c->pool.lastchg, (size_t)c->cfg.pool_slots * 4));
    c->owned.push_back(c->pool.lastchg);
  }
  if (track) HIPCHK(c, hipMemsetAsync(c->pool.lastchg, 0, (size_t)M1 * 4, s));
  if (o.trace) {
    if (!c->pool.tref) {
      HIPCHK(c, hipMalloc(&c->pool.tref, (size_t)c->cfg.pool_slots * 8));
      c->owned.push_back(c->pool.tref);
      HIPCHK(c, hipMalloc(&c->d_trace_n, 256));
      c->owned.push_back(c->d_trace_n);
    }
    if (tcap > c->trace_alloc) {
      if (c->d_trace_rec) {
        HIPCHK(c, hipStreamSynchronize(s));
        HIPCHK(c, hipFree(c->d_trace_rec));
        c->owned.erase(std::find(c->owned.begin(), c->owned.end(), (void *)c->d_trace_rec));
        c->d_trace_rec = nullptr;
        c->trace_alloc = 0;
      }
      HIPCHK(c, hipMalloc(&c->d_trace_rec, (size_t)tcap * 8));
      c->owned.push_back(c->d_trace_rec);
      c->trace_alloc = tcap;
    }
    HIPCHK(c, hipMemsetAsync(c->pool.tref, 0xff, (size_t)c->cfg.pool_slots * 8, s));
    HIPCHK(c, hipMemsetAsync(c->d_trace_n, 0, 4, s));
  }
  c->trace_count = 0;
  int32_t gate_off = 0, gate_words = 0;
  if (o.mode == TRS_MODE_LEARNED) {
    // the predictor's decision table, evaluated on the device for every
    // input, goes right after the rule tables
    if (!c->d_pred) {
      const size_t P = (size_t)TRS_MLP_MAX_SYM * TRS_MLP_EMB + 4096;
      HIPCHK(c, hipMalloc(&c->d_pred, P * 2));
      HIPCHK(c, hipMalloc(&c->d_arity, TRS_MLP_MAX_SYM * 4));
      HIPCHK(c, hipMalloc(&c->d_pprobs, (size_t)TRS_MLP_MAX_SYM * 512 * 4));
      HIPCHK(c, hipMalloc(&c->d_prec, (size_t)TRS_MLP_MAX_SYM * 512 * 8));
      HIPCHK(c, hipMalloc(&c->d_ploss, 256));
      for (void *q : {(void *)c->d_pred, (void *)c->d_arity, (void *)c->d_pprobs,
                      (void *)c->d_prec, (void *)c->d_ploss})
        c->owned.push_back(q);
      c->pred_dirty = true;
    }
    if (c->pred_dirty) {
      HIPCHK(c, hipMemcpyAsync(c->d_pred, c->pred.data(), c->pred.size() * 2,
                               hipMemcpyHostToDevice, s));
      HIPCHK(c, hipMemcpyAsync(c->d_arity, c->arity.data(), c->n_sym * 4,
                               hipMemcpyHostToDevice, s));
      HIPCHK(c, hipStreamSynchronize(s));  // the host vectors may change later
      c->pred_dirty = false;
    }
    gate_off = (int32_t)((c->tab.size() + 3) & ~(size_t)3);
    gate_words = c->n_sym * 16;
    HIPCHK(c, trs_mlp_build_table(c->d_pred, c->n_sym, c->d_arity, o.threshold, c->d_pprobs,
                                  c->d_prec, c->d_ploss, (uint32_t *)(c->d_tab + gate_off), s));
  }

  RoundArgs ra;
  std::memset(&ra, 0, sizeof(ra));  // compared byte-wise with the captured arguments
  ra.p = c->pool;
  ra.ctl = c->d_ctl;
  ra.tab = c->d_tab;
  ra.tab_words = gate_words ? gate_off + gate_words : (int32_t)c->tab.size();
  ra.gate_off = gate_off;
  ra.use_memo = o.trace ? 0 : 1;
  // (0 = the default, -1 = off; the plain mode is the paper's one level per
  // round)
  auto opt = [](int32_t v, int32_t dflt) { return v == 0 ? dflt : std::max(0, v); };
  const bool plain = o.mode == TRS_MODE_PLAIN;
  ra.nf_walk = plain ? 0 : opt(o.nf_walk, TRS_DEFAULT_WALK);
  ra.nf_walk_wide = plain ? 0 : opt(o.nf_walk_wide, TRS_DEFAULT_WALK_WIDE);
  ra.cont_passes = ra.nf_walk ? opt(o.cont_passes, TRS_DEFAULT_CONT) : 0;
  ra.cont_passes_wide = ra.nf_walk_wide ? std::max(0, o.cont_passes_wide) : 0;
  ra.fresh_below = (int32_t)(c->cfg.pool_slots * o.place_fresh / 100);
  // learned mode's periodic full sweeps (off by default): dropped nodes are
  // woken by parent notification, and a round that makes no progress is
  // followed by a full sweep, so these only bound how long a missed wake-up
  // could wait (on the 4096-term batch, before the walk: 5.4 s every 8
  // rounds, 3.4 s every 64)
  ra.sweep_every = o.mode == TRS_MODE_LEARNED ? std::max(0, o.sweep_every) : 0;
  if (o.trace) {
    ra.label_h = o.label_horizon > 0 ? o.label_horizon : 1;
    ra.trace_rate = (uint32_t)o.trace;
    ra.trace_cap_rec = tcap;
    ra.trace_rec = c->d_trace_rec;
    ra.trace_n = c->d_trace_n;
  }
  ra.n_sym = c->n_sym;
  ra.n_rules = c->n_rules;
  ra.npt = npt;
  ra.bar = c->d_bar;
  ra.mode = o.mode;
  // opt-in phase trace of workgroup 0 (TRS_PHASE_TRACE=path: the first
  // rounds' timestamps are written there as text after the run)
  const char *trace_path = std::getenv("TRS_PHASE_TRACE");
  long long *d_trace = nullptr;
  const int trace_cap = 4096;
  // TRS_PHASE_MAX set: a row per traced round and workgroup (the first 64)
  const bool trace_wg = trace_path && std::getenv("TRS_PHASE_MAX") != nullptr;
  const size_t trace_rows = (size_t)trace_cap * (trace_wg ? 64 : 1);
  const size_t trace_bytes = trace_rows * TRACE_FIELDS * 8;
  if (trace_path) {
    HIPCHK(c, hipMalloc(&d_trace, trace_bytes));
    HIPCHK(c, hipMemsetAsync(d_trace, 0, trace_bytes, s));
    ra.trace = d_trace;
    ra.trace_cap = trace_cap;
    // TRS_PHASE_SHIFT=s samples rounds r with r mod 2^s < 2 over the whole run
    if (const char *sh = std::getenv("TRS_PHASE_SHIFT")) ra.trace_shift = std::atoi(sh);
    ra.trace_max = trace_wg;
  }
  // opt-in per-workgroup timing of one round (TRS_WG_TRACE=round:path)
  const char *wgt_env = std::getenv("TRS_WG_TRACE");
  long long *d_wgt = nullptr;
  std::string wgt_path;
  if (wgt_env) {
    const char *colon = std::strchr(wgt_env, ':');
    if (colon) {
      ra.wgtrace_round = std::atoi(wgt_env);
      wgt_path = colon + 1;
      HIPCHK(c, hipMalloc(&d_wgt, 4096 * 8 * 8));
      HIPCHK(c, hipMemsetAsync(d_wgt, 0, 4096 * 8 * 8, s));
      ra.wgtrace = d_wgt;
    }
  }
  // LDS list buffers: four entries per thread for small workgroups, two for
  // large ones (whose LDS goes to the sweep); with 16 slots per thread the
  // sweep copies tiles ahead into an LDS ring, as deep (up to 4) as fits
  ra.qbuf = B >= 512 ? 2 : 4;
  ra.pf_depth = 0;
  if (npt == 16 && o.pf_depth >= 0) {
    const int want = o.pf_depth > 0 ? o.pf_depth : 4;
    for (int d = want; d >= 1; d--) {
      if (trs_round_lds_bytes(B, npt, ra.tab_words, c->n_rules, d, ra.qbuf) <= 160 * 1024) {
        ra.pf_depth = d;
        break;
      }
    }
  }
  const size_t lds = trs_round_lds_bytes(B, npt, ra.tab_words, c->n_rules, ra.pf_depth, ra.qbuf);
  if (lds > 160 * 1024) return c->fail(TRS_E_ARG, "configuration needs too much LDS");
  const int TILE = B * npt;
  HIPCHK(c, trs_prepare_kernels(A, lds));
  int gmax = o.max_grid > 0 ? o.max_grid : 8 * c->cu_count;
  if (!o.persistent) {
    // The grid of a round launch stays within what the chip holds at once,
    // so that every workgroup is dispatched, and reads the published line,
    // at the launch's start.  A workgroup dispatched only after the working
    // ones had finished (one that had to wait for a free slot) would read
    // the line the last of them published for the next launch, and could
    // run that round a second time.
    const int res = trs_round_resident(A, B, lds, c->cfg.device);
    if (res > 0) gmax = std::min(gmax, res);
  }
  if (o.persistent) {
    gmax = trs_max_resident(A, B, lds, c->cfg.device);
    if (gmax <= 0) return c->fail(TRS_E_HIP, "persistent kernel cannot be resident");
  }
  // grid sizes are powers of two (at least 8 when large enough) so that the
  // captured chunk is re-captured only when the slot extent doubles
  auto grid_for = [&](int64_t n) {
    int64_t need = std::max<int64_t>(1, (n + TILE - 1) / TILE);
    int64_t g = 1;
    while (g < need) g <<= 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, gmax));
  };
  int64_t r = 0, n_est = M1, launches = 0;
  const int K = 64;        // launches per captured chunk (each runs >= 1 round)
  int P = 1;               // chunks (or persistent launches) per poll
  const int KP = o.rounds_per_poll ? o.rounds_per_poll : 64;  // persistent rounds per launch
  // one workgroup runs rounds alone while their lists hold at most this
  // many items (one pass of the workgroup: on the 4096-term batch a launch
  // beats two or more passes of one workgroup, 2.62 s against 2.75 s at
  // four), continuing for up to cont_rounds rounds inside one launch
  ra.small_cap = B;
  // plain mode: large full rounds are classified by k_scan, launched before
  // each round launch, and run as list rounds (not in the persistent form,
  // nor when tracing; TRS_NO_SCAN=1 keeps the sweep inside k_round).  On the
  // 4096-term batch: 5.4 s against 6.3 s for the in-kernel sweep.
  ra.use_scan = (o.mode == TRS_MODE_PLAIN && !o.persistent && ra.use_memo &&
                 std::getenv("TRS_NO_SCAN") == nullptr) ? 1 : 0;
  ra.round_block = B;
  // the scan's lists: 16 (each of N/8 entries, 8 in each frontier buffer)
  // for pools of 2^24 slots or more, whose lists then hold every slot a
  // list's workgroups can list (at most n/16 + 2^19 + 2^10 for grids of at
  // most 512); else one list of N entries
  {
    const int64_t N = c->cfg.pool_slots;
    ra.scan_lists = N >= (int64_t)1 << 24 ? 16 : 1;
    ra.scan_rs = ra.scan_lists == 16 ? N / 8 : N;
  }
  // the scan grid: a workgroup per scan tile, at most 2 per compute unit
  auto scan_grid_for = [&](int64_t n) {
    const int64_t ts = (int64_t)SCAN_BLOCK * SCAN_NPT;
    int64_t need = std::max<int64_t>(1, (n + ts - 1) / ts);
    int64_t g = 1;
    while (g < need) g <<= 1;
    return (int)std::min<int64_t>(g, std::min<int64_t>(512, 2 * (int64_t)std::max(1, c->cu_count)));
  };
  ra.cont_rounds = 4096;
  ra.max_rounds = o.max_rounds;
  HIPCHK(c, hipEventRecord(c->ev0, s));
  const size_t small = offsetof(Ctl, stat);  // control words and round counters
  // opt-in progress lines on stderr for long runs (TRS_PROGRESS set)
  const bool progress = std::getenv("TRS_PROGRESS") != nullptr;
  const auto t_start = std::chrono::steady_clock::now();
  double last_report = 0.0;
  int64_t front_est = 0;
  // the launches skip a round whose lists or sweep a grid four times larger
  // would still take in four passes (k_round, k_scan: grid_too_small): the
  // estimates above come from the last poll, and a term that grows fast
  // (a tree that doubles every round) would otherwise run many rounds on a
  // grid sized for its first.  An interval that made no progress raises the
  // grid (at least doubling it, so the loop ends); one that did lowers that
  // floor again.
  int g_floor = 1;
  int64_t r_polled = -1;
  int g_prev = -1, sg_prev = -1;  // the previous interval's launch shape
  trs_status result = TRS_OK;
  for (;;) {
    int g = grid_for(n_est);
    if (o.mode == TRS_MODE_FRONTIER && front_est > 0) {
      // frontier rounds need only as many workgroups as queued items (twice
      // the last observed count, as a power of two; a list takes a pass per
      // B items, a sweep one per B * npt slots, so this may exceed the sweep's
      // grid); the rare full sweeps stride over all tiles with the same grid.
      // A persistent grid also pays its device-wide barrier per workgroup.
      // (Learned mode keeps the full grid: its periodic sweeps are frequent.)
      int64_t need = std::max<int64_t>(8, (2 * front_est + B - 1) / B);
      int64_t gg = 1;
      while (gg < need) gg <<= 1;
      g = (int)std::min<int64_t>(gg, gmax);
    }
    g = std::min(gmax, std::max(g, g_floor));
    if (o.persistent || g >= gmax) {
      ra.grow_list = ra.grow_full = 0;
    } else {
      const int64_t gl = (int64_t)g * B * 4, gf = (int64_t)g * TILE * 4;
      ra.grow_list = gl <= INT32_MAX ? (int)gl : 0;
      ra.grow_full = gf <= INT32_MAX ? (int)gf : 0;
    }
    if (o.persistent) {
      for (int i = 0; i < P; i++) {
        HIPCHK(c, hipMemcpyAsync(c->d_bar, c->h_zero, 8, hipMemcpyHostToDevice, s));
        ra.nrounds = KP;
        HIPCHK(c, trs_launch_persistent(A, ra, g, B, s));
        launches++;
      }
    } else {
      const int sg = ra.use_scan ? scan_grid_for(n_est) : 0;
      const bool cached = c->gexec && c->g_grid == g && c->g_sgrid == sg && c->g_block == B &&
                          c->g_k == K && c->g_lds == lds &&
                          std::memcmp(&c->g_args, &ra, sizeof(ra)) == 0;
      // a launch shape is captured once the previous interval used it too:
      // while the grid still changes from poll to poll (a term that grows
      // fast) plain launches cost less than a capture per interval
      const bool stable = g == g_prev && sg == sg_prev;
      g_prev = g;
      sg_prev = sg;
      if (!cached && !stable) {
        for (int i = 0; i < P * K; i++) {
          if (ra.use_scan) HIPCHK(c, trs_launch_scan(A, ra, sg, s));
          HIPCHK(c, trs_launch_round(A, ra, g, B, s));
        }
        launches += (int64_t)P * K;
      } else {
        if (!cached) {
          if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
          if (c->graph) (void)hipGraphDestroy(c->graph);
          c->gexec = nullptr;
          c->graph = nullptr;
          HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
          for (int k = 0; k < K; k++) {
            hipError_t e = ra.use_scan ? trs_launch_scan(A, ra, sg, s) : hipSuccess;
            if (e == hipSuccess) e = trs_launch_round(A, ra, g, B, s);
            if (e != hipSuccess) {
              hipGraph_t junk;
              (void)hipStreamEndCapture(s, &junk);
              return c->fail(TRS_E_HIP, std::string("capture: ") + hipGetErrorString(e));
            }
          }
          HIPCHK(c, hipStreamEndCapture(s, &c->graph));
          HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
          c->g_grid = g;
          c->g_sgrid = sg;
          c->g_block = B;
          c->g_k = K;
          c->g_lds = lds;
          std::memcpy(&c->g_args, &ra, sizeof(ra));
        }
        for (int i = 0; i < P; i++) {
          HIPCHK(c, hipGraphLaunch(c->gexec, s));
          launches += K;
        }
      }
    }
    HIPCHK(c, hipMemcpyAsync(c->h_ctl, c->d_ctl, small, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    r = c->h_ctl->r_cur;
    if (progress) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      if (el - last_report >= 10.0) {
        std::fprintf(stderr, "[trs] round %lld, extent %d, %.0f s\n", (long long)r,
                     c->h_ctl->peak_n, el);
        last_report = el;
      }
    }
    if (c->h_ctl->abort) {
      result = c->fail(TRS_E_INTERNAL, "device-wide barrier timed out");
      break;
    }
    if (c->h_ctl->done) break;
    // (the device stops the run at round max_rounds itself; this only guards
    // a run whose device state is inconsistent)
    if (o.max_rounds > 0 && r > o.max_rounds + 1) {
      result = c->fail(TRS_E_ROUNDS, "no normal form within max_rounds");
      break;
    }
    // the extent at the start of the last issued round, and of the round
    // published for the next launch
    n_est = std::max<int64_t>(n_est, std::max(c->h_ctl->peak_n, c->h_ctl->pub[3]));
    front_est = 0;
    for (int k = 0; k < 3; k++)
      front_est = std::max<int64_t>(front_est, c->h_ctl->cnt[k].front + c->h_ctl->cnt[k].dead);
    if (r == r_polled) {
      // no round ran: the grid was too small for the published round
      int64_t want = 2 * (int64_t)g, need_pub = std::max(1, c->h_ctl->pub[2]), p2 = 1;
      while (p2 < need_pub) p2 <<= 1;
      g_floor = (int)std::min<int64_t>(gmax, std::max(want, p2));
      P = 1;
      if (progress) std::fprintf(stderr, "[trs] round %lld: grid %d -> at least %d\n",
                                 (long long)r, g, g_floor);
    } else {
      g_floor = std::max(1, g_floor / 2);
      P = std::min(P * 2, o.rounds_per_poll ? 1 : 64);
    }
    r_polled = r;
  }
  HIPCHK(c, hipEventRecord(c->ev1, s));
  HIPCHK(c, hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (d_wgt) {
    std::vector<long long> t(4096 * 8);
    HIPCHK(c, hipMemcpy(t.data(), d_wgt, t.size() * 8, hipMemcpyDeviceToHost));
    (void)hipFree(d_wgt);
    if (FILE *f = std::fopen(wgt_path.c_str(), "w")) {
      for (int i = 0; i < 4096; i++) {
        if (!t[i * 8]) continue;
        std::fprintf(f, "%d", i);
        for (int j = 0; j < 8; j++) std::fprintf(f, " %lld", t[i * 8 + j]);
        std::fprintf(f, "\n");
      }
      std::fclose(f);
    }
  }
  if (d_trace) {
    std::vector<long long> t(trace_rows * TRACE_FIELDS);
    HIPCHK(c, hipMemcpy(t.data(), d_trace, t.size() * 8, hipMemcpyDeviceToHost));
    (void)hipFree(d_trace);
    // one line per round (workgroup 0), or per round and workgroup ("row wg
    // fields", rows with a timestamp only)
    if (FILE *f = std::fopen(trace_path, "w")) {
      for (size_t i = 0; i < trace_rows; i++) {
        const long long *v = &t[i * TRACE_FIELDS];
        if (trace_wg) {
          bool any = false;
          for (int j = 0; j < TRACE_FIELDS; j++) any |= v[j] != 0;
          if (!any) continue;
          std::fprintf(f, "%zu %zu", i / 64, i % 64);
        } else {
          std::fprintf(f, "%zu", i);
        }
        for (int j = 0; j < TRACE_FIELDS; j++) std::fprintf(f, " %lld", v[j]);
        std::fprintf(f, "\n");
      }
      std::fclose(f);
    }
  }
  const Ctl &h = *c->h_ctl;
  c->stamp_base += (int32_t)std::min<int64_t>(r + 2, 1 << 30);
  if (o.trace) {
    int32_t nt = 0;
    HIPCHK(c, hipMemcpy(&nt, c->d_trace_n, 4, hipMemcpyDeviceToHost));
    c->trace_count = std::min<int64_t>(nt, tcap);
  }
  if (result == TRS_OK && h.err) {
    result = c->fail(h.err, h.err == TRS_E_POOL     ? "node pool exhausted during rewriting"
                            : h.err == TRS_E_ROUNDS ? "no normal form within max_rounds"
                                                    : "device reported an inconsistency");
  }
  for (int i = 0; i < c->n_rules; i++) {
    unsigned long long t = 0;
    for (int j = 0; j < RULE_SPREAD; j++) t += h.rule_apps[j][i];
    c->rule_counts[i] = (int64_t)t;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    auto sum = [&](int k) {
      unsigned long long t = 0;
      for (int j = 0; j < CTL_SPREAD; j++) t += h.stat[j][k];
      return (int64_t)t;
    };
    stats->rounds = h.done ? h.done_round : r;
    for (int64_t v : c->rule_counts) stats->rule_apps += v;
    stats->node_visits = sum(STAT_VISITS);
    stats->active_visits = sum(STAT_ACTIVE);
    stats->allocs = sum(STAT_ALLOC);
    stats->frees = sum(STAT_FREED);
    stats->peak_slots = h.peak_n;
    stats->gc_rounds = h.gc_rounds;
    stats->mlp_evals = sum(STAT_MLP);
    stats->full_sweeps = h.full_sweeps;
    stats->launches = launches;
    stats->ready_visits = sum(STAT_READY);
    stats->nf_set = sum(STAT_NFSET);
    stats->rc_atomics = sum(STAT_RCOPS);
    stats->memo_blocked = sum(STAT_MEMO);
    stats->mlp_kept = sum(STAT_KEEP);
    stats->trace_records = sum(STAT_TRACE);
    stats->nf_walked = sum(STAT_WALK);
    stats->last_progress_round = h.last_prog;
    stats->device_ms = ms;
  }
  if (result != TRS_OK) return result;
  c->n_final = h.n_final;
  c->fs_final[0] = h.fs_final[0];
  c->fs_final[1] = h.fs_final[1];
  c->normalized = true;
  return TRS_OK;
}

trs_status trs_read_nf(trs_ctx *c, int32_t term_id, int32_t *buf, int64_t cap, int64_t *len_out) {
  if (!c || !len_out) return TRS_E_ARG;
  if (!c->normalized) return c->fail(TRS_E_STATE, "normalize first");
  if (term_id < 0 || term_id >= c->n_terms) return c->fail(TRS_E_ARG, "bad term id");
  const int A = c->A;
  if (!c->cache_valid) {
    const int64_t n = c->n_final;
    c->c_hss.resize(n);
    c->c_args.resize((size_t)n * A);
    c->c_state.resize(n);
    HIPCHK(c, hipMemcpy(c->c_hss.data(), c->pool.hss, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(c->c_args.data(), c->pool.args, n * A * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(c->c_state.data(), c->pool.state, n, hipMemcpyDeviceToHost));
    c->cache_valid = true;
  }
  const int64_t n = c->n_final;
  std::vector<int32_t> stk;
  stk.push_back(c->roots[term_id]);
  int64_t len = 0;
  while (!stk.empty()) {
    int32_t x = stk.back();
    stk.pop_back();
    if (x <= 0 || x >= n) return c->fail(TRS_E_INTERNAL, "dangling argument index");
    if (!(c->c_state[x] & ST_NF)) return c->fail(TRS_E_INTERNAL, "reachable node not in normal form");
    int32_t s = c->c_hss[x];
    if (s < 0 || s >= c->n_sym) return c->fail(TRS_E_INTERNAL, "bad symbol in pool");
    if (buf) {
      if (len >= cap) return c->fail(TRS_E_ARG, "buffer too small");
      buf[len] = s;
    }
    len++;
    if (len > INT32_MAX) return c->fail(TRS_E_LIMIT, "normal form too long");
    for (int j = c->arity[s] - 1; j >= 0; j--) stk.push_back(c->c_args[(size_t)x * A + j]);
  }
  *len_out = len;
  return TRS_OK;
}

trs_status trs_autotune(trs_ctx *c, const trs_opts *base, trs_opts *best, trs_tune_result *res) {
  if (!c || !base || !best) return TRS_E_ARG;
  if (!c->terms_loaded) return c->fail(TRS_E_STATE, "load rules and terms first");
  trs_tune_result r;
  std::memset(&r, 0, sizeof(r));
  auto it = c->tuned.find(base->mode);
  if (it != c->tuned.end()) {
    *best = *base;
    best->block = it->second.block;
    best->nodes_per_thread = it->second.npt;
    best->max_grid = it->second.grid;
    r.best_block = best->block;
    r.best_npt = best->nodes_per_thread;
    r.best_grid = best->max_grid;
    r.best_ms = it->second.ms;
    if (res) *res = r;
    return TRS_OK;
  }
  Tuned bt{0, 16, 0, 0.0};
  auto trial = [&](int B, int npt, int grid) -> trs_status {
    trs_opts o = *base;
    o.block = B;
    o.nodes_per_thread = npt;
    o.max_grid = grid;
    trs_stats st;
    const trs_status s = trs_normalize(c, &o, &st);
    if (s != TRS_OK) return s;
    const int k = r.trials++;
    r.block[k] = B;
    r.npt[k] = npt;
    r.grid[k] = grid;
    r.ms[k] = st.device_ms;
    if (bt.block == 0 || st.device_ms < bt.ms) bt = Tuned{B, npt, grid, st.device_ms};
    return TRS_OK;
  };
  // Block sizes first at 16 nodes per thread, then the other nodes per
  // thread at the best block: a staged walk over the block x nodes-per-
  // thread grid.  In plain mode the scan kernel classifies the large full
  // rounds, so the round kernel's shape matters for the list rounds that
  // follow (narrow workgroups spread the examined slots over more compute
  // units) and for small pools swept inside it; 1024-thread workgroups,
  // which only slow the list rounds, are left out there.
  const bool plain = base->mode == TRS_MODE_PLAIN;
  for (int B : {64, 128, 256, 512, 1024}) {
    if (plain && B > 512) continue;
    const trs_status s = trial(B, 16, 0);
    if (s != TRS_OK) return s;
  }
  const int B0 = bt.block;
  for (int npt : {1, 2, 4, 8}) {
    if (plain && npt == 1) continue;
    const trs_status s = trial(B0, npt, 0);
    if (s != TRS_OK) return s;
  }
  c->tuned[base->mode] = bt;
  *best = *base;
  best->block = bt.block;
  best->nodes_per_thread = bt.npt;
  best->max_grid = bt.grid;
  r.best_block = bt.block;
  r.best_npt = bt.npt;
  r.best_grid = bt.grid;
  r.best_ms = bt.ms;
  if (res) *res = r;
  return TRS_OK;
}

trs_status trs_set_predictor(trs_ctx *c, const uint16_t *params_bf16, int64_t n_params) {
  if (!c || !params_bf16) return TRS_E_ARG;
  if (!c->rules_loaded) return c->fail(TRS_E_STATE, "load rules first");
  const int64_t P = trs_mlp_param_count(c->n_sym);
  if (P < 0) return c->fail(TRS_E_LIMIT, "learned mode supports at most 256 symbols");
  if (n_params != P) return c->fail(TRS_E_ARG, "parameter count does not match the system");
  c->pred.assign(params_bf16, params_bf16 + P);
  c->pred_dirty = true;
  return TRS_OK;
}

trs_status trs_read_trace(trs_ctx *c, uint64_t *buf, int64_t cap, int64_t *n_out) {
  if (!c || !n_out) return TRS_E_ARG;
  if (!c->normalized) return c->fail(TRS_E_STATE, "normalize first");
  const int64_t n = c->trace_count;
  if (!buf) {
    *n_out = n;
    return TRS_OK;
  }
  if (cap < 0) return c->fail(TRS_E_ARG, "negative capacity");
  const int64_t k = std::min(n, cap);
  if (k > 0)
    HIPCHK(c, hipMemcpy(buf, c->d_trace_rec, (size_t)k * 8, hipMemcpyDeviceToHost));
  *n_out = k;
  return TRS_OK;
}

trs_status trs_read_pool(trs_ctx *c, trs_pool_info *info, int32_t *hss, int32_t *args,
                         uint8_t *state, int32_t *rc, int32_t *free0, int32_t *free1,
                         int32_t *roots) {
  if (!c || !info) return TRS_E_ARG;
  if (!c->normalized) return c->fail(TRS_E_STATE, "normalize first");
  const int64_t n = c->n_final, A = c->A;
  info->n = n;
  info->maxarity = (int32_t)A;
  info->n_terms = c->n_terms;
  info->free0 = c->fs_final[0];
  info->free1 = c->fs_final[1];
  if (info->free0 < 0 || info->free1 < 0 || info->free0 > c->cfg.pool_slots ||
      info->free1 > c->cfg.pool_slots)
    return c->fail(TRS_E_INTERNAL, "free-stack sizes out of range");
  const hipStream_t s = c->stream;
  HIPCHK(c, hipStreamSynchronize(s));
  if (hss) HIPCHK(c, hipMemcpy(hss, c->pool.hss, n * 4, hipMemcpyDeviceToHost));
  if (args) HIPCHK(c, hipMemcpy(args, c->pool.args, n * A * 4, hipMemcpyDeviceToHost));
  if (state) HIPCHK(c, hipMemcpy(state, c->pool.state, n, hipMemcpyDeviceToHost));
  if (rc) HIPCHK(c, hipMemcpy(rc, c->pool.rc, n * 4, hipMemcpyDeviceToHost));
  if (free0 && info->free0)
    HIPCHK(c, hipMemcpy(free0, c->pool.fstack0, info->free0 * 4, hipMemcpyDeviceToHost));
  if (free1 && info->free1)
    HIPCHK(c, hipMemcpy(free1, c->pool.fstack1, info->free1 * 4, hipMemcpyDeviceToHost));
  if (roots)
    for (int32_t t = 0; t < c->n_terms; t++) roots[t] = c->roots[t];
  return TRS_OK;
}

trs_status trs_rule_counts(trs_ctx *c, int64_t *out, int32_t cap) {
  if (!c || !out) return TRS_E_ARG;
  if (!c->normalized) return c->fail(TRS_E_STATE, "normalize first");
  if (cap < c->n_rules) return c->fail(TRS_E_ARG, "buffer too small");
  for (int i = 0; i < c->n_rules; i++) out[i] = c->rule_counts[i];
  return TRS_OK;
}

}  // extern "C"
