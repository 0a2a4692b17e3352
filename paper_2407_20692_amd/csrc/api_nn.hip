// C ABI of the learned denoiser (declared in include/cpi.h): the network's
// layer table, parameter layout and workspace plan, its forward pass and
// training step, the image-quality measures, and single-kernel entry points
// that expose every kernel of the network on its own.
//
// The network is a four-level convolutional encoder-decoder (widths 32, 64,
// 128, 256; two 3x3 convolutions with ReLU per level; 2x2 max-pooling down,
// nearest 2x upsampling and concatenation with the encoder output up; a 1x1
// output convolution), applied as x + f(x) to planes normalised by their own
// mean and standard deviation.  Every convolution is a BF16 matrix-core
// implicit GEMM with FP32 sums; master weights and Adam moments are FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <exception>
#include <mutex>
#include <string>
#include <utility>

#include "cpi.h"
#include "errors.h"
#include "kernels.h"

namespace {

using cpi::report_error;

cpi_status bad(const std::string& m) { return report_error(CPI_ERR_INVALID_ARG, m); }

template <typename F>
cpi_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::exception& e) {
    return report_error(CPI_ERR_DEVICE, std::string("internal error: ") + e.what());
  } catch (...) {
    return report_error(CPI_ERR_DEVICE, "internal error");
  }
}

#define NN_HIP(call, what)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return report_error(CPI_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---- layer table ---------------------------------------------------------------
struct Layer {
  const char* name;
  int cin, cout, ks;        // as stored (channel counts padded for the kernels)
  int cin_used, cout_used;  // logical channels
  int level;                // resolution level 0..3 (size H >> level)
};

constexpr int kNumLayers = 15;
// gradient buffers of the backward pass, taken in turn: the chain of input
// gradients may run this many steps ahead of the weight gradients that read
// its results
constexpr int kGradBufs = 6;
const Layer kLayers[kNumLayers] = {
    {"enc1a", 8, 32, 3, 1, 32, 0},     {"enc1b", 32, 32, 3, 32, 32, 0},
    {"enc2a", 32, 64, 3, 32, 64, 1},   {"enc2b", 64, 64, 3, 64, 64, 1},
    {"enc3a", 64, 128, 3, 64, 128, 2}, {"enc3b", 128, 128, 3, 128, 128, 2},
    {"mid_a", 128, 256, 3, 128, 256, 3}, {"mid_b", 256, 256, 3, 256, 256, 3},
    {"dec3a", 384, 128, 3, 384, 128, 2}, {"dec3b", 128, 128, 3, 128, 128, 2},
    {"dec2a", 192, 64, 3, 192, 64, 1}, {"dec2b", 64, 64, 3, 64, 64, 1},
    {"dec1a", 96, 32, 3, 96, 32, 0},   {"dec1b", 32, 32, 3, 32, 32, 0},
    {"out", 32, 32, 1, 32, 1, 0},
};
enum { ENC1A, ENC1B, ENC2A, ENC2B, ENC3A, ENC3B, MIDA, MIDB, DEC3A, DEC3B, DEC2A, DEC2B, DEC1A,
       DEC1B, OUT };

struct Params {
  int64_t w_off[kNumLayers], b_off[kNumLayers], total = 0;          // FP32 master layout
  int kpad[kNumLayers], kpad_t[kNumLayers];
  int64_t wf_off[kNumLayers], wt_off[kNumLayers], packed_total = 0;  // BF16 packed layout
};

Params param_layout() {
  Params p;
  int64_t off = 0, pk = 0;
  for (int i = 0; i < kNumLayers; ++i) {
    const Layer& L = kLayers[i];
    const int64_t taps = int64_t(L.ks) * L.ks;
    p.w_off[i] = off;
    off = round_up(off + L.cout * taps * L.cin, 64);
    p.b_off[i] = off;
    off = round_up(off + L.cout, 64);
    p.kpad[i] = int(round_up(taps * L.cin, 32));
    p.kpad_t[i] = int(round_up(taps * L.cout, 32));
    p.wf_off[i] = pk;
    pk = round_up(pk + int64_t(L.cout) * p.kpad[i], 128);
    p.wt_off[i] = pk;
    pk = round_up(pk + int64_t(L.cin) * p.kpad_t[i], 128);
  }
  p.total = off;
  p.packed_total = pk;
  return p;
}

// ---- workspace plan --------------------------------------------------------------
struct Net {
  uint16_t* x8;
  uint16_t* act[kNumLayers - 1];  // outputs of the ReLU layers
  uint16_t* pool[3];
  uint16_t* cat[3];
  float* outf;       // the network's output channel [P0], FP32
  float* opart;      // partial sums of the output layer's gradients
  float* xf;
  float* tn;
  float* stats;
  double* norm_scratch;
  float* loss_scratch;
  uint16_t* g[kGradBufs];  // gradient buffers, taken in turn by the backward pass
  uint16_t* skip[3];
  uint16_t* wpack;
  float* grads;
  float* wpart[2];   // partial sums of the weight gradients' pixel splits (two,
                     // used in turn, so one layer's reduction can overlap the
                     // next layer's kernel)
  int64_t wpart_cap; // floats at each wpart
  size_t bytes;
};

// Lays the buffers out from base (null: sizes only).
Net plan_net(uint8_t* base, int B, int H, int W, bool train) {
  Net n{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void* p = base ? base + off : nullptr;
    off = size_t(round_up(int64_t(off + bytes), 256));
    return p;
  };
  const int64_t P0 = int64_t(B) * H * W;
  auto P = [&](int level) { return P0 >> (2 * level); };
  const Params pl = param_layout();
  n.x8 = static_cast<uint16_t*>(take(size_t(P0) * 8 * 2));
  for (int i = 0; i < kNumLayers - 1; ++i)
    n.act[i] = static_cast<uint16_t*>(take(size_t(P(kLayers[i].level)) * kLayers[i].cout * 2));
  const int wid[4] = {32, 64, 128, 256};
  for (int l = 0; l < 3; ++l) {
    n.pool[l] = static_cast<uint16_t*>(take(size_t(P(l + 1)) * wid[l] * 2));
    n.cat[l] = static_cast<uint16_t*>(take(size_t(P(l)) * (wid[l + 1] + wid[l]) * 2));
  }
  n.outf = static_cast<float*>(take(size_t(P0) * 4));
  n.xf = static_cast<float*>(take(size_t(P0) * 4));
  n.stats = static_cast<float*>(take(size_t(B) * 2 * 4));
  n.norm_scratch = static_cast<double*>(take(cpi::nn_normalize_scratch_bytes(B)));
  n.wpack = static_cast<uint16_t*>(take(size_t(pl.packed_total) * 2));
  if (train) {
    n.tn = static_cast<float*>(take(size_t(P0) * 4));
    n.opart = static_cast<float*>(take(size_t(cpi::nn_out1_bwd_groups(P0)) * 36 * 4));
    n.loss_scratch = static_cast<float*>(take(64));
    for (int k = 0; k < kGradBufs; ++k) n.g[k] = static_cast<uint16_t*>(take(size_t(P0) * 96 * 2));
    for (int l = 0; l < 3; ++l) n.skip[l] = static_cast<uint16_t*>(take(size_t(P(l)) * wid[l] * 2));
    n.grads = static_cast<float*>(take(size_t(pl.total) * 4));
    int64_t cap = 0;
    for (int i = 0; i < kNumLayers; ++i) {
      const Layer& L = kLayers[i];
      cpi::NnWgradArgs w;
      w.B = B;
      w.H = H >> L.level;
      w.W = W >> L.level;
      w.Cin = L.cin;
      w.Cout = L.cout;
      w.ks = L.ks;
      w.Kpad = pl.kpad[i];
      const int64_t f = i == ENC1A ? int64_t(cpi::nn_in1_wgrad_groups(P0)) *
                                         (int64_t(32) * 9 * L.cin + 32)
                                   : cpi::nn_conv_wgrad_part_floats(w);
      if (f > cap) cap = f;
    }
    n.wpart_cap = cap;
    for (int k = 0; k < 2; ++k) n.wpart[k] = static_cast<float*>(take(size_t(cap) * 4));
  }
  n.bytes = off;
  return n;
}

cpi_status check_net_shape(int B, int H, int W) {
  if (B < 1 || H < 8 || W < 8 || H % 8 || W % 8)
    return bad("denoiser planes need batch >= 1 and H, W positive multiples of 8");
  if (int64_t(B) * H * W > (int64_t(1) << 26))
    return bad("denoiser batch too large: batch * H * W must not exceed 2^26");
  return CPI_OK;
}

// ---- weight-gradient streams -----------------------------------------------------
// The backward pass runs each layer's weight gradient on a second stream of
// the device, and the reduction of its partial sums on a third (both one per
// device, made at first use, default priority), so that they overlap the
// chain of input gradients on the caller's stream and each other.  Events
// order the streams: each host thread keeps its own events per device.
constexpr int kSideEvents = 96;
std::mutex g_side_mu;
hipStream_t g_side_stream[64] = {};
hipStream_t g_red_stream[64] = {};
thread_local hipEvent_t t_side_ev[64][kSideEvents] = {};

hipError_t side_resources(const void* ws, hipStream_t* side, hipStream_t* red, hipEvent_t** ev) {
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, ws);
  if (e != hipSuccess) return e;
  const int dev = at.device;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (!g_side_stream[dev] || !g_red_stream[dev] || !t_side_ev[dev][kSideEvents - 1]) {
    int cur = 0;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    e = hipSetDevice(dev);
    if (e != hipSuccess) return e;
    {
      std::lock_guard<std::mutex> lk(g_side_mu);
      if (!g_side_stream[dev]) e = hipStreamCreateWithFlags(&g_side_stream[dev], hipStreamNonBlocking);
      if (e == hipSuccess && !g_red_stream[dev])
        e = hipStreamCreateWithFlags(&g_red_stream[dev], hipStreamNonBlocking);
    }
    for (int k = 0; k < kSideEvents && e == hipSuccess; ++k)
      if (!t_side_ev[dev][k]) e = hipEventCreateWithFlags(&t_side_ev[dev][k], hipEventDisableTiming);
    const hipError_t e2 = hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
  }
  *side = g_side_stream[dev];
  *red = g_red_stream[dev];
  *ev = t_side_ev[dev];
  return hipSuccess;
}

// ---- network passes --------------------------------------------------------------
// The input gradient of a decoder level's first layer, split as its input
// [upsample2(low) (c1 channels), skip]: dlow (summed over the four copies,
// zeroed where mask <= 0) and dskip.
struct GradSplit {
  uint16_t* dlow;
  uint16_t* dskip;
  const uint16_t* mask;
  int c1;
};

struct Pass {
  const Params& pl;
  const Net& n;
  const float* params;
  int B, H, W;
  hipStream_t s;
  hipStream_t side = nullptr;  // weight-gradient stream, or null: all on s
  hipStream_t red = nullptr;   // their reductions' stream (set with side)
  hipEvent_t* ev = nullptr;    // kSideEvents events for ordering the streams
  int* nev = nullptr;          // events used so far
  hipEvent_t* pfree = nullptr; // [2]: the reduction that last read n.wpart[k], or null
  int* pnext = nullptr;        // the partial buffer the next weight gradient takes
  float* loss = nullptr;       // the loss is added here by backward()

  int hl(int level) const { return H >> level; }
  int wl(int level) const { return W >> level; }
  int64_t P(int level) const { return int64_t(B) * hl(level) * wl(level); }

  cpi::NnConvArgs conv_args(int i) const {
    const Layer& L = kLayers[i];
    cpi::NnConvArgs a;
    a.B = B;
    a.H = hl(L.level);
    a.W = wl(L.level);
    a.Cin = L.cin;
    a.Cout = L.cout;
    a.ks = L.ks;
    a.Kpad = pl.kpad[i];
    return a;
  }

  // whether layer i's convolution reads its input as [upsampled low (c_low
  // channels), in] without the concatenation being written out
  bool reads_concat(int i, int c_low) const {
    cpi::NnConvArgs a = conv_args(i);
    a.c_low = c_low;
    return cpi::nn_conv_takes_low(a);
  }

  // input: in, or [upsample2(low) (c_low channels), in] when low is set, or
  // the 2x2 max-pooling of in when pool_in
  hipError_t conv(int i, const uint16_t* in, uint16_t* out, float* out_f32, bool relu,
                  const uint16_t* low = nullptr, int c_low = 0, bool pool_in = false) const {
    const Layer& L = kLayers[i];
    if (i == ENC1A && relu && out && !out_f32)
      return cpi::nn_in1_fwd(in, B, hl(L.level), wl(L.level), L.cin, n.wpack + pl.wf_off[i],
                             pl.kpad[i], params + pl.b_off[i], out, s);
    cpi::NnConvArgs a = conv_args(i);
    a.in = in;
    a.wk = n.wpack + pl.wf_off[i];
    a.bias = params + pl.b_off[i];
    a.out = out;
    a.out_f32 = out_f32;
    a.relu = relu ? 1 : 0;
    a.low = low;
    a.c_low = low ? c_low : 0;
    a.pool_in = pool_in ? 1 : 0;
    return cpi::nn_conv(a, s);
  }

  // layer i (ReLU output into out) on the 2x2 max-pooling of the encoder
  // output n.act[2 * lv + 1] (level lv), read in place when the kernel can,
  // else pooled into n.pool[lv] first
  hipError_t conv_pooled(int i, int lv, uint16_t* out) const {
    cpi::NnConvArgs a = conv_args(i);
    a.pool_in = 1;
    if (cpi::nn_conv_takes_low(a)) return conv(i, n.act[2 * lv + 1], out, nullptr, true, nullptr, 0, true);
    const int wid[4] = {32, 64, 128, 256};
    hipError_t e = cpi::nn_maxpool(n.act[2 * lv + 1], B, hl(lv), wl(lv), wid[lv], n.pool[lv], s);
    if (e != hipSuccess) return e;
    return conv(i, n.pool[lv], out, nullptr, true);
  }

  // weight and bias gradients of layer i (on the weight-gradient stream when
  // there is one: it waits for the caller's stream up to here, and *done is
  // recorded after it); input gradient into gin (masked by `mask` if given)
  // unless gin is null, on the caller's stream
  // With split, gin is scratch for the whole input gradient when the
  // convolution cannot write it split itself.
  hipError_t back(int i, const uint16_t* in, const uint16_t* g, uint16_t* gin,
                  const uint16_t* mask, hipEvent_t* done = nullptr, const uint16_t* low = nullptr,
                  int c_low = 0, bool pool_in = false, const GradSplit* split = nullptr) const {
    const Layer& L = kLayers[i];
    hipStream_t ws = s;
    hipError_t e;
    if (side) {
      const hipEvent_t ready = ev[(*nev)++];
      if ((e = hipEventRecord(ready, s)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(side, ready, 0)) != hipSuccess) return e;
      ws = side;
    }
    cpi::NnWgradArgs w;
    w.in = in;
    w.dy = g;
    w.dw = n.grads + pl.w_off[i];
    w.B = B;
    w.H = hl(L.level);
    w.W = wl(L.level);
    w.Cin = L.cin;
    w.Cout = L.cout;
    w.ks = L.ks;
    w.Kpad = pl.kpad[i];
    w.db = n.grads + pl.b_off[i];
    w.part_cap = n.wpart_cap;
    w.low = low;
    w.c_low = low ? c_low : 0;
    w.pool_in = pool_in ? 1 : 0;
    const bool in1 = i == ENC1A && !gin;
    auto run = [&](hipStream_t st, int phases) {
      return in1 ? cpi::nn_in1_wgrad(in, B, w.H, w.W, L.cin, g, w.part, w.dw, w.db, st, phases)
                 : cpi::nn_conv_wgrad(w, st, phases);
    };
    if (!side) {
      w.part = n.wpart[0];
      if ((e = run(s, 3)) != hipSuccess) return e;
    } else {
      // partial buffer k in turn, once the reduction that last read it is done
      const int k = *pnext;
      *pnext ^= 1;
      if (pfree[k]) {
        if ((e = hipStreamWaitEvent(side, pfree[k], 0)) != hipSuccess) return e;
        pfree[k] = nullptr;
      }
      w.part = n.wpart[k];
      if ((e = run(side, 1)) != hipSuccess) return e;
      const hipEvent_t wdone = ev[(*nev)++];
      if ((e = hipEventRecord(wdone, side)) != hipSuccess) return e;
      if (done) *done = wdone;  // the kernel that read g
      if ((e = hipStreamWaitEvent(red, wdone, 0)) != hipSuccess) return e;
      if ((e = run(red, 2)) != hipSuccess) return e;
      pfree[k] = ev[(*nev)++];
      if ((e = hipEventRecord(pfree[k], red)) != hipSuccess) return e;
    }
    if (!gin) return hipSuccess;
    cpi::NnConvArgs a;
    a.in = g;
    a.wk = n.wpack + pl.wt_off[i];
    a.mask = mask;
    a.out = gin;
    a.B = B;
    a.H = hl(L.level);
    a.W = wl(L.level);
    a.Cin = L.cout;
    a.Cout = L.cin;
    a.ks = L.ks;
    a.Kpad = pl.kpad_t[i];
    if (split) {
      cpi::NnConvArgs sa = a;
      sa.out = nullptr;
      sa.mask = nullptr;
      sa.dlow = split->dlow;
      sa.dskip = split->dskip;
      sa.low_mask = split->mask;
      sa.c1 = split->c1;
      if (cpi::nn_conv_takes_split(sa)) return cpi::nn_conv(sa, s);
      if ((e = cpi::nn_conv(a, s)) != hipSuccess) return e;
      return cpi::nn_upcat_grad(gin, B, a.H / 2, a.W / 2, split->c1, a.Cout - split->c1, split->mask,
                                split->dlow, split->dskip, s);
    }
    return cpi::nn_conv(a, s);
  }

  hipError_t pack(bool transposed) const {
    cpi::NnPackTable tab;
    int64_t begin = 0;
    for (int i = 0; i < kNumLayers; ++i) {
      const Layer& L = kLayers[i];
      cpi::NnPackLayer& d = tab.layer[i];
      d.w_off = pl.w_off[i];
      d.wf_off = pl.wf_off[i];
      d.wt_off = pl.wt_off[i];
      d.cout = L.cout;
      d.cin = L.cin;
      d.ks = L.ks;
      d.kpad = pl.kpad[i];
      d.kpad_t = pl.kpad_t[i];
      d.transposed = transposed && i != ENC1A;
      d.begin = begin;
      begin += int64_t(L.cout) * d.kpad + (d.transposed ? int64_t(L.cin) * d.kpad_t : 0);
    }
    tab.n = kNumLayers;
    tab.total = begin;
    return cpi::nn_pack_all(params, n.wpack, tab, s);
  }

  hipError_t forward() const {
    hipError_t e;
#define NN_STEP(x)                  \
  do {                              \
    if ((e = (x)) != hipSuccess) return e; \
  } while (0)
    const int wid[4] = {32, 64, 128, 256};
    // encoder: level l's first layer reads the pooled output of level l - 1
    for (int l = 0; l < 3; ++l) {
      if (l == 0) {
        NN_STEP(conv(0, n.x8, n.act[0], nullptr, true));
      } else {
        NN_STEP(conv_pooled(2 * l, l - 1, n.act[2 * l]));
      }
      NN_STEP(conv(2 * l + 1, n.act[2 * l], n.act[2 * l + 1], nullptr, true));
    }
    NN_STEP(conv_pooled(MIDA, 2, n.act[MIDA]));
    NN_STEP(conv(MIDB, n.act[MIDA], n.act[MIDB], nullptr, true));
    const uint16_t* h = n.act[MIDB];
    for (int l = 2; l >= 0; --l) {
      const int da = DEC3A + 2 * (2 - l);
      if (reads_concat(da, wid[l + 1])) {
        NN_STEP(conv(da, n.act[2 * l + 1], n.act[da], nullptr, true, h, wid[l + 1]));
      } else {
        NN_STEP(cpi::nn_upcat(h, n.act[2 * l + 1], B, hl(l + 1), wl(l + 1), wid[l + 1], wid[l],
                              n.cat[l], s));
        NN_STEP(conv(da, n.cat[l], n.act[da], nullptr, true));
      }
      NN_STEP(conv(da + 1, n.act[da], n.act[da + 1], nullptr, true));
      h = n.act[da + 1];
    }
    NN_STEP(cpi::nn_out1_fwd(h, n.wpack + pl.wf_off[OUT], params + pl.b_off[OUT], P(0), n.outf, s));
    return hipSuccess;
  }

  // the loss of the output in n.outf against the targets in n.tn (added to
  // *loss) and its gradients.  Each step writes its result into the next of
  // the kGradBufs gradient buffers; a buffer is taken again kGradBufs steps later,
  // after the caller's stream has waited for the weight gradient that read it.
  hipError_t backward() const {
    hipError_t e;
    const int wid[4] = {32, 64, 128, 256};
    hipEvent_t busy[kGradBufs] = {};
    int cur = 0, nxt = 0;
    auto take = [&](int* b) -> hipError_t {
      *b = nxt;
      nxt = (nxt + 1) % kGradBufs;
      if (busy[*b]) {
        const hipError_t r = hipStreamWaitEvent(s, busy[*b], 0);
        busy[*b] = nullptr;
        return r;
      }
      return hipSuccess;
    };
    // layer i's gradients from the gradient in buffer cur; its input
    // gradient (unless last) into a new buffer, which becomes cur
    auto layer = [&](int i, const uint16_t* in, const uint16_t* mask, bool input_grad,
                     const uint16_t* low = nullptr, int c_low = 0, bool pool_in = false) {
      int b = -1;
      hipError_t r = input_grad ? take(&b) : hipSuccess;
      if (r != hipSuccess) return r;
      r = back(i, in, n.g[cur], input_grad ? n.g[b] : nullptr, mask, &busy[cur], low, c_low,
               pool_in);
      if (input_grad) cur = b;
      return r;
    };
    {
      int b;
      NN_STEP(take(&b));
      NN_STEP(cpi::nn_out1_bwd(n.outf, n.xf, n.tn, P(0), n.act[DEC1B], n.wpack + pl.wf_off[OUT],
                               n.g[b], loss, n.opart, n.grads + pl.w_off[OUT],
                               n.grads + pl.b_off[OUT], s));
      cur = b;
    }
    // decoder, level 0 up to 2: cur holds the gradient of the level's second
    // convolution's pre-activation
    const uint16_t* below[3] = {n.act[DEC2B], n.act[DEC3B], n.act[MIDB]};
    for (int l = 0; l < 3; ++l) {
      const int da = DEC1A - 2 * l;
      NN_STEP(layer(da + 1, n.act[da], n.act[da], true));
      // the input [upsampled level l + 1 output, encoder output] read as
      // such; its gradient written split into dlow (level l + 1) and skip[l]
      int bs, bl;
      NN_STEP(take(&bs));
      NN_STEP(take(&bl));
      const GradSplit sp{n.g[bl], n.skip[l], below[l], wid[l + 1]};
      NN_STEP(back(da, n.act[2 * l + 1], n.g[cur], n.g[bs], nullptr, &busy[cur], below[l],
                   wid[l + 1], false, &sp));
      cur = bl;
    }
    NN_STEP(layer(MIDB, n.act[MIDA], n.act[MIDA], true));
    // the first layer of levels 1 .. 3 reads the pooled encoder output in place
    NN_STEP(layer(MIDA, n.act[ENC3B], nullptr, true, nullptr, 0, true));
    // encoder, level 2 down to 0: cur holds the gradient of the pooled output
    for (int l = 2; l >= 0; --l) {
      uint16_t* yb = n.act[2 * l + 1];
      int b;
      NN_STEP(take(&b));
      NN_STEP(cpi::nn_pool_bwd_add(yb, B, hl(l), wl(l), wid[l], n.g[cur], n.skip[l], n.g[b], s));
      cur = b;
      NN_STEP(layer(2 * l + 1, n.act[2 * l], n.act[2 * l], true));
      if (l == 0) {
        NN_STEP(layer(0, n.x8, nullptr, false));
      } else {
        NN_STEP(layer(2 * l, n.act[2 * l - 1], nullptr, true, nullptr, 0, true));
      }
    }
    if (side) {
      for (hipStream_t st : {side, red}) {
        const hipEvent_t joined = ev[(*nev)++];
        NN_STEP(hipEventRecord(joined, st));
        NN_STEP(hipStreamWaitEvent(s, joined, 0));
      }
    }
    return hipSuccess;
#undef NN_STEP
  }
};

}  // namespace

extern "C" {

cpi_status cpi_denoiser_layer_count(int32_t* count) {
  if (!count) return bad("count is null");
  *count = kNumLayers;
  return CPI_OK;
}

cpi_status cpi_denoiser_layer_info(int32_t index, cpi_denoiser_layer* out) {
  if (!out) return bad("out is null");
  if (index < 0 || index >= kNumLayers) return bad("layer index out of range");
  const Params pl = param_layout();
  const Layer& L = kLayers[index];
  std::memset(out, 0, sizeof(*out));
  std::strncpy(out->name, L.name, sizeof(out->name) - 1);
  out->cin = L.cin;
  out->cout = L.cout;
  out->ks = L.ks;
  out->cin_used = L.cin_used;
  out->cout_used = L.cout_used;
  out->weight_offset = pl.w_off[index];
  out->bias_offset = pl.b_off[index];
  return CPI_OK;
}

cpi_status cpi_denoiser_param_count(int64_t* count) {
  if (!count) return bad("count is null");
  *count = param_layout().total;
  return CPI_OK;
}

cpi_status cpi_denoiser_workspace_size(int32_t batch, int32_t h, int32_t w, int32_t train,
                                       size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!bytes) return bad("bytes is null");
    cpi_status st = check_net_shape(batch, h, w);
    if (st != CPI_OK) return st;
    *bytes = plan_net(nullptr, batch, h, w, train != 0).bytes;
    return CPI_OK;
  });
}

cpi_status cpi_denoiser_forward(const float* params, int32_t batch, int32_t h, int32_t w,
                                const float* planes, float* out, void* workspace,
                                size_t workspace_bytes, void* stream) {
  return guarded([&]() -> cpi_status {
    cpi_status st = check_net_shape(batch, h, w);
    if (st != CPI_OK) return st;
    if (!params || !planes || !out || !workspace) return bad("null device pointer");
    if (!al16(params) || !al16(planes) || !al16(out) || !al16(workspace))
      return bad("device pointers must be 16-byte aligned");
    const Net n = plan_net(static_cast<uint8_t*>(workspace), batch, h, w, false);
    if (workspace_bytes < n.bytes)
      return report_error(CPI_ERR_WORKSPACE, "denoiser workspace too small: need " +
                                                 std::to_string(n.bytes) + " bytes");
    const Params pl = param_layout();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Pass ps{pl, n, params, batch, h, w, s};
    const int64_t hw = int64_t(h) * w;
    NN_HIP(cpi::nn_normalize(planes, batch, hw, 8, n.x8, n.xf, nullptr, nullptr, n.stats,
                             n.norm_scratch, s),
           "denoiser normalise");
    NN_HIP(ps.pack(false), "denoiser weights");
    NN_HIP(ps.forward(), "denoiser forward");
    NN_HIP(cpi::nn_denormalize(n.outf, 1, n.xf, n.stats, hw, batch, out, s), "denoiser output");
    return CPI_OK;
  });
}

cpi_status cpi_denoiser_train_step(float* params, float* adam_m, float* adam_v, int64_t step,
                                   float lr, int32_t batch, int32_t h, int32_t w,
                                   const float* planes, const float* targets, float* loss,
                                   void* workspace, size_t workspace_bytes, void* stream) {
  return guarded([&]() -> cpi_status {
    cpi_status st = check_net_shape(batch, h, w);
    if (st != CPI_OK) return st;
    if (!params || !adam_m || !adam_v || !planes || !targets || !loss || !workspace)
      return bad("null device pointer");
    if (!al16(params) || !al16(adam_m) || !al16(adam_v) || !al16(planes) || !al16(targets) ||
        !al16(workspace))
      return bad("device pointers must be 16-byte aligned");
    if (step < 1) return bad("Adam step numbers start at 1");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return bad("learning rate must be positive and finite");
    const Net n = plan_net(static_cast<uint8_t*>(workspace), batch, h, w, true);
    if (workspace_bytes < n.bytes)
      return report_error(CPI_ERR_WORKSPACE, "denoiser workspace too small: need " +
                                                 std::to_string(n.bytes) + " bytes");
    const Params pl = param_layout();
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStream_t side = nullptr, red = nullptr;
    hipEvent_t* ev = nullptr;
    int nev = 0, pnext = 0;
    hipEvent_t pfree[2] = {nullptr, nullptr};
    NN_HIP(side_resources(workspace, &side, &red, &ev), "denoiser weight-gradient streams");
    const Pass ps{pl, n, params, batch, h, w, s, side, red, ev, &nev, pfree, &pnext, loss};
    const int64_t hw = int64_t(h) * w, P0 = int64_t(batch) * hw;
    NN_HIP(cpi::nn_normalize(planes, batch, hw, 8, n.x8, n.xf, targets, n.tn, n.stats,
                             n.norm_scratch, s),
           "denoiser normalise");
    NN_HIP(ps.pack(true), "denoiser weights");
    NN_HIP(ps.forward(), "denoiser forward");
    NN_HIP(cpi::fill_u32(reinterpret_cast<uint32_t*>(n.grads), pl.total, 0u, s), "denoiser grads");
    NN_HIP(cpi::fill_u32(reinterpret_cast<uint32_t*>(loss), 1, 0u, s), "denoiser loss");
    NN_HIP(ps.backward(), "denoiser backward");
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = float(1.0 - std::pow(b1, double(step)));
    const float c2 = float(1.0 - std::pow(b2, double(step)));
    NN_HIP(cpi::nn_adam(params, n.grads, adam_m, adam_v, pl.total, lr, float(b1), float(b2), 1e-8f,
                        c1, c2, s),
           "denoiser Adam");
    return CPI_OK;
  });
}

cpi_status cpi_denoiser_gradients(const float* params, int32_t batch, int32_t h, int32_t w,
                                  const float* planes, const float* targets, float* loss,
                                  float* grads, void* workspace, size_t workspace_bytes,
                                  void* stream) {
  return guarded([&]() -> cpi_status {
    cpi_status st = check_net_shape(batch, h, w);
    if (st != CPI_OK) return st;
    if (!params || !planes || !targets || !loss || !grads || !workspace)
      return bad("null device pointer");
    if (!al16(params) || !al16(planes) || !al16(targets) || !al16(grads) || !al16(workspace))
      return bad("device pointers must be 16-byte aligned");
    Net n = plan_net(static_cast<uint8_t*>(workspace), batch, h, w, true);
    if (workspace_bytes < n.bytes)
      return report_error(CPI_ERR_WORKSPACE, "denoiser workspace too small: need " +
                                                 std::to_string(n.bytes) + " bytes");
    n.grads = grads;
    const Params pl = param_layout();
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStream_t side = nullptr, red = nullptr;
    hipEvent_t* ev = nullptr;
    int nev = 0, pnext = 0;
    hipEvent_t pfree[2] = {nullptr, nullptr};
    NN_HIP(side_resources(workspace, &side, &red, &ev), "denoiser weight-gradient streams");
    const Pass ps{pl, n, params, batch, h, w, s, side, red, ev, &nev, pfree, &pnext, loss};
    const int64_t hw = int64_t(h) * w, P0 = int64_t(batch) * hw;
    NN_HIP(cpi::nn_normalize(planes, batch, hw, 8, n.x8, n.xf, targets, n.tn, n.stats,
                             n.norm_scratch, s),
           "denoiser normalise");
    NN_HIP(ps.pack(true), "denoiser weights");
    NN_HIP(ps.forward(), "denoiser forward");
    NN_HIP(cpi::fill_u32(reinterpret_cast<uint32_t*>(grads), pl.total, 0u, s), "denoiser grads");
    NN_HIP(cpi::fill_u32(reinterpret_cast<uint32_t*>(loss), 1, 0u, s), "denoiser loss");
    NN_HIP(ps.backward(), "denoiser backward");
    return CPI_OK;
  });
}

cpi_status cpi_image_quality(const float* pred, const float* target, int32_t batch, int32_t h,
                             int32_t w, double* psnr, double* ssim, void* stream) {
  return guarded([&]() -> cpi_status {
    if (batch < 1 || h < 11 || w < 11) return bad("planes must be at least 11 x 11, batch >= 1");
    if (!pred || !target || !psnr || !ssim) return bad("null device pointer");
    NN_HIP(cpi::nn_quality(pred, target, batch, h, w, psnr, ssim, static_cast<hipStream_t>(stream)),
           "image quality");
    return CPI_OK;
  });
}

// ---- single kernels -------------------------------------------------------------------
namespace {
cpi_status check_conv(int32_t b, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t ks) {
  if (b < 1 || h < 1 || w < 1) return bad("sizes must be positive");
  if (cin < 8 || cin % 8) return bad("cin must be a positive multiple of 8");
  if (cout < 32 || cout % 32) return bad("cout must be a positive multiple of 32");
  if (ks != 1 && ks != 3) return bad("ks must be 1 or 3");
  if (int64_t(b) * h * w > (int64_t(1) << 28)) return bad("batch * h * w must not exceed 2^28");
  return CPI_OK;
}
}  // namespace

cpi_status cpi_nn_conv2d(const uint16_t* x, const uint16_t* w_packed, const float* bias,
                         const uint16_t* mask, int32_t relu, int32_t b, int32_t h, int32_t w,
                         int32_t cin, int32_t cout, int32_t ks, int32_t kpad, uint16_t* out,
                         float* out_f32, void* stream) {
  return guarded([&]() -> cpi_status {
    cpi_status st = check_conv(b, h, w, cin, cout, ks);
    if (st != CPI_OK) return st;
    if (kpad != round_up(int64_t(ks) * ks * cin, 32))
      return bad("kpad must be ks*ks*cin rounded up to a multiple of 32");
    if (!x || !w_packed || (!out && !out_f32)) return bad("null device pointer");
    if (!al16(x) || !al16(w_packed)) return bad("x and w_packed must be 16-byte aligned");
    cpi::NnConvArgs a;
    a.in = x;
    a.wk = w_packed;
    a.bias = bias;
    a.mask = mask;
    a.out = out;
    a.out_f32 = out_f32;
    a.B = b;
    a.H = h;
    a.W = w;
    a.Cin = cin;
    a.Cout = cout;
    a.ks = ks;
    a.Kpad = kpad;
    a.relu = relu ? 1 : 0;
    NN_HIP(cpi::nn_conv(a, static_cast<hipStream_t>(stream)), "conv2d");
    return CPI_OK;
  });
}

namespace {
cpi::NnWgradArgs wgrad_args(int32_t b, int32_t h, int32_t w, int32_t cin, int32_t cout,
                            int32_t ks) {
  cpi::NnWgradArgs a;
  a.B = b;
  a.H = h;
  a.W = w;
  a.Cin = cin;
  a.Cout = cout;
  a.ks = ks;
  a.Kpad = int(round_up(int64_t(ks) * ks * cin, 32));
  return a;
}
}  // namespace

cpi_status cpi_nn_conv2d_wgrad_workspace_size(int32_t b, int32_t h, int32_t w, int32_t cin,
                                              int32_t cout, int32_t ks, size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!bytes) return bad("bytes is null");
    cpi_status st = check_conv(b, h, w, cin, cout, ks);
    if (st != CPI_OK) return st;
    *bytes = size_t(cpi::nn_conv_wgrad_part_floats(wgrad_args(b, h, w, cin, cout, ks))) * 4;
    return CPI_OK;
  });
}

cpi_status cpi_nn_conv2d_wgrad(const uint16_t* x, const uint16_t* dy, int32_t b, int32_t h,
                               int32_t w, int32_t cin, int32_t cout, int32_t ks, float* dw,
                               float* db, void* workspace, size_t workspace_bytes,
                               void* stream) {
  return guarded([&]() -> cpi_status {
    cpi_status st = check_conv(b, h, w, cin, cout, ks);
    if (st != CPI_OK) return st;
    if (!x || !dy || !dw) return bad("null device pointer");
    if (!al16(x) || !al16(dy)) return bad("x and dy must be 16-byte aligned");
    cpi::NnWgradArgs a = wgrad_args(b, h, w, cin, cout, ks);
    if (workspace) {
      const int64_t need = cpi::nn_conv_wgrad_part_floats(a);
      if (workspace_bytes < size_t(need) * 4)
        return report_error(CPI_ERR_WORKSPACE, "conv2d wgrad workspace too small: need " +
                                                   std::to_string(need * 4) + " bytes");
      if (!al16(workspace)) return bad("workspace must be 16-byte aligned");
      a.part = static_cast<float*>(workspace);
      a.part_cap = need;
    }
    a.in = x;
    a.dy = dy;
    a.dw = dw;
    a.db = db;
    NN_HIP(cpi::nn_conv_wgrad(a, static_cast<hipStream_t>(stream)), "conv2d wgrad");
    return CPI_OK;
  });
}

cpi_status cpi_nn_pack_weights(const float* w, int32_t cout, int32_t cin, int32_t ks,
                               uint16_t* w_packed, uint16_t* w_packed_t, void* stream) {
  return guarded([&]() -> cpi_status {
    if (cout < 1 || cin < 1 || ks < 1) return bad("sizes must be positive");
    if (!w || !w_packed) return bad("null device pointer");
    const int kpad = int(round_up(int64_t(ks) * ks * cin, 32));
    const int kpad_t = int(round_up(int64_t(ks) * ks * cout, 32));
    NN_HIP(cpi::nn_pack_weights(w, cout, cin, ks, w_packed, kpad, w_packed_t, kpad_t,
                                static_cast<hipStream_t>(stream)),
           "pack weights");
    return CPI_OK;
  });
}

cpi_status cpi_nn_bias_grad(const uint16_t* dy, int64_t pixels, int32_t c, float* db,
                            void* stream) {
  return guarded([&]() -> cpi_status {
    if (pixels < 1 || c < 1) return bad("sizes must be positive");
    if (!dy || !db) return bad("null device pointer");
    NN_HIP(cpi::nn_bias_grad(dy, pixels, c, db, static_cast<hipStream_t>(stream)), "bias grad");
    return CPI_OK;
  });
}

cpi_status cpi_nn_maxpool2(const uint16_t* x, int32_t b, int32_t h, int32_t w, int32_t c,
                           uint16_t* out, void* stream) {
  return guarded([&]() -> cpi_status {
    if (b < 1 || h < 2 || w < 2 || c < 1 || h % 2 || w % 2) return bad("h and w must be even");
    if (!x || !out) return bad("null device pointer");
    NN_HIP(cpi::nn_maxpool(x, b, h, w, c, out, static_cast<hipStream_t>(stream)), "maxpool");
    return CPI_OK;
  });
}

cpi_status cpi_nn_maxpool2_grad(const uint16_t* x, const uint16_t* dout, int32_t b, int32_t h,
                                int32_t w, int32_t c, uint16_t* dx, void* stream) {
  return guarded([&]() -> cpi_status {
    if (b < 1 || h < 2 || w < 2 || c < 1 || h % 2 || w % 2) return bad("h and w must be even");
    if (!x || !dout || !dx) return bad("null device pointer");
    NN_HIP(cpi::nn_maxpool_bwd(x, b, h, w, c, dout, dx, static_cast<hipStream_t>(stream)),
           "maxpool grad");
    return CPI_OK;
  });
}

cpi_status cpi_nn_upsample2(const uint16_t* x, int32_t b, int32_t h, int32_t w, int32_t c,
                            uint16_t* out, void* stream) {
  return guarded([&]() -> cpi_status {
    if (b < 1 || h < 1 || w < 1 || c < 1) return bad("sizes must be positive");
    if (!x || !out) return bad("null device pointer");
    NN_HIP(cpi::nn_upsample(x, b, h, w, c, out, static_cast<hipStream_t>(stream)), "upsample");
    return CPI_OK;
  });
}

cpi_status cpi_nn_upsample2_grad(const uint16_t* dout, int32_t b, int32_t h, int32_t w, int32_t c,
                                 const uint16_t* mask, uint16_t* dx, void* stream) {
  return guarded([&]() -> cpi_status {
    if (b < 1 || h < 1 || w < 1 || c < 1) return bad("sizes must be positive");
    if (!dout || !dx) return bad("null device pointer");
    NN_HIP(cpi::nn_upsample_bwd(dout, b, h, w, c, mask, dx, static_cast<hipStream_t>(stream)),
           "upsample grad");
    return CPI_OK;
  });
}

cpi_status cpi_nn_upsample2_concat(const uint16_t* low, const uint16_t* skip, int32_t b, int32_t h,
                                  int32_t w, int32_t c1, int32_t c2, uint16_t* out, void* stream) {
  return guarded([&]() -> cpi_status {
    if (b < 1 || h < 1 || w < 1 || c1 < 8 || c2 < 8 || c1 % 8 || c2 % 8)
      return bad("sizes must be positive and channel counts multiples of 8");
    if (!low || !skip || !out) return bad("null device pointer");
    if (!al16(low) || !al16(skip) || !al16(out)) return bad("pointers must be 16-byte aligned");
    NN_HIP(cpi::nn_upcat(low, skip, b, h, w, c1, c2, out, static_cast<hipStream_t>(stream)),
           "upsample concat");
    return CPI_OK;
  });
}

cpi_status cpi_nn_upsample2_concat_grad(const uint16_t* d, int32_t b, int32_t h, int32_t w,
                                       int32_t c1, int32_t c2, const uint16_t* mask,
                                       uint16_t* dlow, uint16_t* dskip, void* stream) {
  return guarded([&]() -> cpi_status {
    if (b < 1 || h < 1 || w < 1 || c1 < 8 || c2 < 8 || c1 % 8 || c2 % 8)
      return bad("sizes must be positive and channel counts multiples of 8");
    if (!d || !dlow || !dskip) return bad("null device pointer");
    if (!al16(d) || !al16(dlow) || !al16(dskip) || (mask && !al16(mask)))
      return bad("pointers must be 16-byte aligned");
    NN_HIP(cpi::nn_upcat_grad(d, b, h, w, c1, c2, mask, dlow, dskip,
                              static_cast<hipStream_t>(stream)),
           "upsample concat grad");
    return CPI_OK;
  });
}

cpi_status cpi_nn_concat(const uint16_t* a, const uint16_t* b, int64_t pixels, int32_t ca,
                         int32_t cb, uint16_t* out, void* stream) {
  return guarded([&]() -> cpi_status {
    if (pixels < 1 || ca < 1 || cb < 1) return bad("sizes must be positive");
    if (!a || !b || !out) return bad("null device pointer");
    NN_HIP(cpi::nn_concat(a, b, pixels, ca, cb, out, static_cast<hipStream_t>(stream)), "concat");
    return CPI_OK;
  });
}

cpi_status cpi_nn_split(const uint16_t* d, int64_t pixels, int32_t ca, int32_t cb, uint16_t* da,
                        uint16_t* db, void* stream) {
  return guarded([&]() -> cpi_status {
    if (pixels < 1 || ca < 1 || cb < 1) return bad("sizes must be positive");
    if (!d || !da || !db) return bad("null device pointer");
    NN_HIP(cpi::nn_split(d, pixels, ca, cb, da, db, static_cast<hipStream_t>(stream)), "split");
    return CPI_OK;
  });
}

cpi_status cpi_nn_add_mask(uint16_t* x, const uint16_t* add, const uint16_t* mask, int64_t count,
                           void* stream) {
  return guarded([&]() -> cpi_status {
    if (count < 1) return bad("count must be positive");
    if (!x) return bad("null device pointer");
    NN_HIP(cpi::nn_add_mask(x, add, mask, count, static_cast<hipStream_t>(stream)), "add mask");
    return CPI_OK;
  });
}

cpi_status cpi_nn_mse(const float* y, int32_t c, const float* residual, const float* target,
                      int64_t pixels, float* loss, uint16_t* dy, void* stream) {
  return guarded([&]() -> cpi_status {
    if (pixels < 1 || c < 1) return bad("sizes must be positive");
    if (!y || !target) return bad("null device pointer");
    NN_HIP(cpi::nn_mse(y, c, residual, target, pixels, loss, dy, static_cast<hipStream_t>(stream)),
           "mse");
    return CPI_OK;
  });
}

cpi_status cpi_nn_adam(float* w, const float* g, float* m, float* v, int64_t count, int64_t step,
                       float lr, float beta1, float beta2, float eps, void* stream) {
  return guarded([&]() -> cpi_status {
    if (count < 1 || step < 1) return bad("count and step must be positive");
    if (!w || !g || !m || !v) return bad("null device pointer");
    const float c1 = float(1.0 - std::pow(double(beta1), double(step)));
    const float c2 = float(1.0 - std::pow(double(beta2), double(step)));
    NN_HIP(cpi::nn_adam(w, g, m, v, count, lr, beta1, beta2, eps, c1, c2,
                        static_cast<hipStream_t>(stream)),
           "adam");
    return CPI_OK;
  });
}

}  // extern "C"
