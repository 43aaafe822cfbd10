// C ABI of the MERA hot path: argument checks, workspace layout and the
// contraction schedules of the ascending / descending superoperators and the
// environments, run on the contraction engine (contract.hip, contract_b3.hip).
//
// Network (one causal cone; Sec. II.B, Fig. 4).  Leg labels used below:
//   fine legs, ket p q r s, bra P Q R S (dimension din)
//   upper legs of the two disentanglers, ket a b | c d, bra A B | C D (din)
//   outer legs of the side isometries x, y (din; traced between ket and bra)
//   coarse legs, ket i j k, bra I J K (dout)
// Ket tensors: uL = u[p q a b], uR = u[r s c d], wL = w[x a i], wC = w[b c j],
// wR = w[d y k]; bra tensors are the same with capital letters except the
// traced fine leg (s for the left window, p for the right window) and x, y.
// Left window: fine legs (p q r | P Q R), s traced.  Right window:
// (q r s | Q R S), p traced.
//
// Schedule of D (both placements share the first three steps):
//   Lp[a i A I] = w[x a i] w[x A I]          Rp[d k D K] = w[d y k] w[D y K]
//   X1[a j k A J K] = Lp . rho               X[j a d A D J] = X1 . Rp       (chi^8)
//   N[r s b d j] = w[b c j] u[r s c d]       M[p q c a j] = u[p q a b] w[b c j]
//   left :  Y = N . X  (sum d j)  -> [r s b a A D J]                          chi^9
//           Z = Y . N' (sum s D J, N' = N with bra legs) -> [r a b A B R]     chi^9
//           W1 = Z . uL (sum a b) -> [p q r A B R];  D_L = W1 . uL' (A B)    chi^8
//   right:  T1 = M . X (sum a j) -> [p q c d A D J]                          chi^9
//           ZR = T1 . M' (sum p A J) -> [q c d D C Q]                         chi^9
//           W2 = ZR . uR (sum c d) -> [q r s C D Q]; D_R = W2 . uR' (C D)    chi^8
// A runs the same steps in reverse (adjoint) order; the environments are the
// reverse-mode derivatives of e = tr(h D(rho)) with respect to the ket copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mera.h"
#include "engine.h"

// Workspace of mera_descend_noalloc: a static device array that every device
// the library runs on holds until the process ends.  In host code `scratch`
// is only a handle for hipGetSymbolAddress, never a device address.
constexpr size_t kNoAllocScratchBytes = size_t(MERA_NOALLOC_SCRATCH_MIB) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_last_error;

void set_err(const std::string& s) { g_last_error = s; }

struct ProfRec {
  std::string step;
  int arith = 0;
  int op = 0;
  double flops = 0.0;
  hipEvent_t a = nullptr, b = nullptr;
};
thread_local bool g_prof_on = false;
thread_local std::vector<ProfRec> g_prof;
thread_local int g_prof_op = -1;  // mera_op of the entry point running on this thread

// Tags the contraction launches of one entry point in the profile records.
struct OpTag {
  int prev;
  explicit OpTag(int op) : prev(g_prof_op) { g_prof_op = op; }
  ~OpTag() { g_prof_op = prev; }
};

using mera::Arith;
using mera::LabelDims;

// Bump allocator over the caller's workspace; in dry mode it only measures.
struct Ctx {
  Arith ar = Arith::F64;
  LabelDims dims;
  hipStream_t s = nullptr;
  bool dry = true;
  char* base = nullptr;
  size_t off = 0;
  double flops = 0.0;
  hipError_t err = hipSuccess;
  double* scratch = nullptr;  // split-k partial sums (see contract())
  size_t scratch_elems = 0;
  std::vector<std::string>* plans = nullptr;  // dry mode: kernel choice of every contraction

  size_t elem() const { return ar == Arith::F64 ? 8 : 4; }
  // reserve `count` elements of `bytes_per` bytes, 256-byte aligned (split
  // tensors, the 4-byte elements of the split-bf16 path, in whole 8-element groups)
  void* take(size_t count, size_t bytes_per) {
    if (ar == Arith::B3 && bytes_per == 4) count = (count + 7) & ~size_t(7);
    off = (off + 255) & ~size_t(255);
    void* p = dry ? nullptr : base + off;
    off += count * bytes_per;
    return p;
  }
  void* take_t(size_t count) { return take(count, elem()); }
  double* take_d(size_t count) { return static_cast<double*>(take(count, 8)); }

  // C = alpha * A . B + beta * C   (A, B of the working type; C of the working type or double)
  void c(const void* A, const char* la, const void* B, const char* lb, void* C, const char* lc,
         bool c_f64, double alpha, double beta, const LabelDims* cdims = nullptr) {
    if (dry) {
      flops += mera::contract_flops(dims, la, lb, lc);
      if (plans)
        plans->push_back(std::string(la) + "," + lb + "->" + lc + " " +
                         mera::contract_plan(ar, dims, la, lb, lc, ar == Arith::F64 || c_f64,
                                             scratch_elems, cdims));
      return;
    }
    if (err != hipSuccess) return;
    const bool cf = (ar == Arith::F64) ? true : c_f64;
    ProfRec rec;
    if (g_prof_on) {
      rec.step = std::string(la) + "," + lb + "->" + lc;
      rec.arith = (int)ar;
      rec.op = g_prof_op;
      rec.flops = mera::contract_flops(dims, la, lb, lc);
      if (hipEventCreate(&rec.a) != hipSuccess || hipEventCreate(&rec.b) != hipSuccess ||
          hipEventRecord(rec.a, s) != hipSuccess) {
        if (rec.a) (void)hipEventDestroy(rec.a);
        if (rec.b) (void)hipEventDestroy(rec.b);
        err = hipErrorOutOfMemory;
        set_err("profile event creation failed");
        return;
      }
    }
    err = mera::contract(ar, dims, A, la, B, lb, C, lc, cf, alpha, beta, s, &flops, scratch,
                         scratch_elems, cdims);
    if (g_prof_on) {
      if (hipEventRecord(rec.b, s) == hipSuccess) {
        g_prof.push_back(rec);
      } else {
        (void)hipEventDestroy(rec.a);
        (void)hipEventDestroy(rec.b);
        if (err == hipSuccess) err = hipErrorInvalidHandle;
        set_err("profile event record failed");
      }
    }
    if (err != hipSuccess)
      set_err(std::string("contract ") + la + "," + lb + "->" + lc + ": " + hipGetErrorString(err));
  }
  void check(hipError_t e, const char* what) {
    if (dry || err != hipSuccess) return;
    if (e != hipSuccess) {
      err = e;
      set_err(std::string(what) + ": " + hipGetErrorString(e));
    }
  }
};

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

// p + n, for buffers that are null in the measuring pass (which takes no
// workspace memory): an offset from a null pointer stays null.
template <class T>
T* advance(T* p, int64_t n) {
  return p ? p + n : nullptr;
}
const void* byte_offset(const void* p, int64_t bytes) {
  return advance(static_cast<const char*>(p), bytes);
}

// Layer tensors in the working type (converted copies for F32; split tensors for B3).
struct LayerT {
  const void* u;
  const void* w;
};

LayerT working_layer(Ctx& cx, const mera_layer* L) {
  const int64_t din = L->din, dout = L->dout;
  if (cx.ar == Arith::F64) return {L->u_d, L->w_d};
  float* uf = static_cast<float*>(cx.take(ipow(din, 4), 4));
  float* wf = static_cast<float*>(cx.take(din * din * dout, 4));
  if (!cx.dry) {
    const bool sp = cx.ar == Arith::B3;
    cx.check(mera::launch_to_f32(L->u_d, uf, ipow(din, 4), sp, cx.s), "to_f32(u)");
    cx.check(mera::launch_to_f32(L->w_d, wf, din * din * dout, sp, cx.s), "to_f32(w)");
  }
  return {uf, wf};
}

// A dout^6 / din^6 FP64 operand in the working type.
const void* working_op(Ctx& cx, const double* x, int64_t n) {
  if (cx.ar == Arith::F64) return x;
  float* xf = static_cast<float*>(cx.take(n, 4));
  if (!cx.dry) cx.check(mera::launch_to_f32(x, xf, n, cx.ar == Arith::B3, cx.s), "to_f32(op)");
  return xf;
}

// Layouts for the split-bf16 path (see Pieces and x_copies).
bool k_contiguous_layouts(const Ctx& cx) { return cx.ar == Arith::B3; }

// A dout^6 density in the working type, with its labels: the split-bf16 path
// moves the legs of the first fine-grained window pair (i, I) innermost, the
// legs the first contraction of every chain sums over.
struct WorkingRho {
  const void* p;
  const char* l;
};
WorkingRho working_rho(Ctx& cx, const double* rho, int64_t dout) {
  if (!k_contiguous_layouts(cx)) return {working_op(cx, rho, ipow(dout, 6)), "ijkIJK"};
  float* y = static_cast<float*>(cx.take(ipow(dout, 6), 4));
  if (!cx.dry) cx.check(mera::launch_rho_to_split_perm(rho, y, (int32_t)dout, cx.s), "rho_to_split");
  return {y, "jkJKiI"};
}

void set_dims(Ctx& cx, int din, int dout) {
  cx.dims = LabelDims();
  cx.dims.set("pqrsPQRSabcdABCDxy", din);
  cx.dims.set("ijkIJK", dout);
  // split-k scratch: 16 partial copies of the largest small-output contraction
  // (din^4 * dout elements), in double
  cx.scratch_elems = (size_t)16 * (size_t)ipow(din, 4) * (size_t)dout;
  cx.scratch = cx.take_d(cx.scratch_elems);
}

// Shared small tensors of one layer.
// N and M appear in several layouts so that every chi^9 contraction sums over
// legs that are contiguous (in the same order) in both of its operands.  The
// split-bf16 path keeps N3 and M3 with those legs innermost ("k-contiguous"),
// which lets its large-tile kernel load both operands straight into LDS.
struct Pieces {
  void *Lp, *Rp;
  void* N;   // [r s b d j]
  void* N3;  // [r b s d j]; split bf16: [s d j r b]
  void* M;   // [p q c a j]
  void* M1;  // [q p c j a]
  void* M3;  // [p c q a j]; split bf16: [p a j c q]
  const char* n3;  // labels of N3 as (R B s D J) legs
  const char* m3;  // labels of M3 as (p C Q A J) legs
  const char* lp;  // labels of Lp: [a i A I]; split bf16: [a A i I]
  const char* rp;  // labels of Rp: [d k D K]; split bf16: [d D k K]
  const char* x1;  // labels of X1 = Lp . rho: [a j k A J K]; split bf16: [a j A J k K]
};

Pieces build_pieces(Ctx& cx, const LayerT& t, int64_t din, int64_t dout) {
  Pieces pc;
  pc.Lp = cx.take_t(din * din * dout * dout);
  pc.Rp = cx.take_t(din * din * dout * dout);
  pc.N = cx.take_t(ipow(din, 4) * dout);
  pc.N3 = cx.take_t(ipow(din, 4) * dout);
  pc.M = cx.take_t(ipow(din, 4) * dout);
  pc.M1 = cx.take_t(ipow(din, 4) * dout);
  pc.M3 = cx.take_t(ipow(din, 4) * dout);
  const bool kc = k_contiguous_layouts(cx);
  pc.lp = kc ? "aAiI" : "aiAI";
  pc.rp = kc ? "dDkK" : "dkDK";
  pc.x1 = kc ? "ajAJkK" : "ajkAJK";
  cx.c(t.w, "xai", t.w, "xAI", pc.Lp, pc.lp, false, 1.0, 0.0);
  cx.c(t.w, "dyk", t.w, "DyK", pc.Rp, pc.rp, false, 1.0, 0.0);
  cx.c(t.w, "bcj", t.u, "rscd", pc.N, "rsbdj", false, 1.0, 0.0);
  cx.c(t.w, "bcj", t.u, "rscd", pc.N3, kc ? "sdjrb" : "rbsdj", false, 1.0, 0.0);
  pc.n3 = kc ? "sDJRB" : "RBsDJ";
  pc.m3 = kc ? "pAJCQ" : "pCQAJ";
  cx.c(t.u, "pqab", t.w, "bcj", pc.M, "pqcaj", false, 1.0, 0.0);
  cx.c(t.u, "pqab", t.w, "bcj", pc.M1, "qpcja", false, 1.0, 0.0);
  cx.c(t.u, "pqab", t.w, "bcj", pc.M3, kc ? "pajcq" : "pcqaj", false, 1.0, 0.0);
  return pc;
}

// X[j a d A D J] = sum Lp[a i A I] rho[i j k I J K] Rp[d k D K]; keeps X1 = Lp.rho.
// with_x = false skips X when only the k-contiguous copies are needed.  The
// dout^4-row operand comes first (the m side of the large-tile kernel).
void build_x(Ctx& cx, const Pieces& pc, const WorkingRho& rho, void* X1, void* X, bool with_x) {
  cx.c(rho.p, rho.l, pc.Lp, pc.lp, X1, pc.x1, false, 1.0, 0.0);
  if (with_x) cx.c(X1, pc.x1, pc.Rp, pc.rp, X, "djaADJ", false, 1.0, 0.0);
}

// Copies of X for the first chi^9 contraction of each chain, with the summed
// legs innermost: [a A D J d j] (left chain, sums d j) and [d D A J j a]
// (right chain, sums j a).  Without them X's summed legs come first and the
// contraction's second operand is contiguous along its output legs.
struct XCopies {
  const void* l;  // labels xl
  const void* r;  // labels xr
  const char* xl;
  const char* xr;
};

XCopies x_copies(Ctx& cx, const Pieces& pc, const void* X1, const void* X, int64_t din,
                 int64_t dout) {
  if (!k_contiguous_layouts(cx)) return {X, X, "djaADJ", "djaADJ"};
  void* xl = cx.take_t(ipow(din, 4) * dout * dout);
  void* xr = cx.take_t(ipow(din, 4) * dout * dout);
  cx.c(X1, pc.x1, pc.Rp, pc.rp, xl, "aADJdj", false, 1.0, 0.0);
  cx.c(X1, pc.x1, pc.Rp, pc.rp, xr, "dDAJja", false, 1.0, 0.0);
  return {xl, xr, "aADJdj", "dDAJja"};
}

struct Bufs {
  void* big;   // din^6 * dout
  void* mid;   // din^6
  void* mid2;  // din^6
};

// `rows` = extent of the sliced leading leg (din when not sliced)
Bufs take_bufs(Ctx& cx, int64_t din, int64_t dout, int64_t rows) {
  Bufs b;
  b.big = cx.take_t(rows * ipow(din, 5) * dout);
  b.mid = cx.take_t(rows * ipow(din, 5));
  b.mid2 = cx.take_t(rows * ipow(din, 5));
  return b;
}

// ---------------------------------------------------------------------------
// D
// ---------------------------------------------------------------------------
// `slices` > 1 processes the left chain in slices of its open leg r (fine
// site 3) and the right chain in slices of q (fine site 2): the chi^7
// intermediates then only need 1/slices of their full size.
int run_descend(Ctx& cx, const mera_layer* L, const double* rho_in, double* rho_out,
                int placement, int slices = 1) {
  const int64_t din = L->din, dout = L->dout;
  set_dims(cx, (int)din, (int)dout);
  LayerT t = working_layer(cx, L);
  const WorkingRho rho = working_rho(cx, rho_in, dout);
  Pieces pc = build_pieces(cx, t, din, dout);
  void* X1 = cx.take_t(din * din * ipow(dout, 4));
  const bool kc = k_contiguous_layouts(cx);
  void* X = kc ? nullptr : cx.take_t(ipow(din, 4) * dout * dout);
  // chi^6 intermediates of the chains; the split-bf16 path stores each with
  // the legs the next contraction sums over innermost
  const char* mid_l = kc ? "rABRab" : "rabABR";
  const char* mid2_l = kc ? "pqrRAB" : "pqrABR";
  const char* mid_r = kc ? "qDCQcd" : "qcdDCQ";
  const char* mid2_r = kc ? "qrsQCD" : "qrsCDQ";
  const int64_t R = (din + slices - 1) / slices;
  build_x(cx, pc, rho, X1, X, !kc);
  const XCopies xc = x_copies(cx, pc, X1, X, din, dout);
  Bufs b = take_bufs(cx, din, dout, R);
  const double wgt = placement == MERA_AVG ? 0.5 : 1.0;
  const LabelDims full = cx.dims;
  const size_t es = cx.elem();
  bool first = true;
  if (placement != MERA_RIGHT) {
    for (int64_t r0 = 0; r0 < din; r0 += R) {
      cx.dims = full;
      cx.dims.d['r'] = std::min(R, din - r0);
      const void* n_s = byte_offset(pc.N, r0 * ipow(din, 3) * dout * es);  // N[r0, ...]
      cx.c(n_s, "rsbdj", xc.l, xc.xl, b.big, "rsbaADJ", false, 1.0, 0.0);
      cx.c(b.big, "rsbaADJ", pc.N, "RsBDJ", b.mid, mid_l, false, 1.0, 0.0);
      cx.c(b.mid, mid_l, t.u, "pqab", b.mid2, mid2_l, false, 1.0, 0.0);
      cx.c(b.mid2, mid2_l, t.u, "PQAB", advance(rho_out, r0 * ipow(din, 3)), "pqrPQR", true, wgt, 0.0, &full);
    }
    cx.dims = full;
    first = false;
  }
  if (placement != MERA_LEFT) {
    for (int64_t q0 = 0; q0 < din; q0 += R) {
      cx.dims = full;
      cx.dims.d['q'] = std::min(R, din - q0);
      const void* m_s = byte_offset(pc.M1, q0 * ipow(din, 3) * dout * es);  // M1[q0, ...]
      cx.c(m_s, "qpcja", xc.r, xc.xr, b.big, "pqcdDAJ", false, 1.0, 0.0);
      cx.c(b.big, "pqcdDAJ", pc.M, "pQCAJ", b.mid, mid_r, false, 1.0, 0.0);
      cx.c(b.mid, mid_r, t.u, "rscd", b.mid2, mid2_r, false, 1.0, 0.0);
      cx.c(b.mid2, mid2_r, t.u, "RSCD", advance(rho_out, q0 * ipow(din, 5)), "qrsQRS", true, wgt,
           first ? 0.0 : 1.0, &full);
    }
    cx.dims = full;
  }
  return 0;
}

// Rows of the sliced leg per slice must be a multiple of this: a slice of the
// split-bf16 pieces N and M1 (din^3 * dout elements per row) has to start on a
// whole 8-element group of the split tensor.
int64_t slice_row_multiple(Arith ar, int64_t din, int64_t dout) {
  if (ar != Arith::B3) return 1;
  const int64_t e = din * din * din * dout;
  return e % 8 == 0 ? 1 : e % 4 == 0 ? 2 : e % 2 == 0 ? 4 : 8;
}

// Slice count with the fewest slices allowed by slice_row_multiple (din
// unsliced rows when even that is not possible).
int max_slices(Arith ar, int64_t din, int64_t dout) {
  const int64_t r = slice_row_multiple(ar, din, dout);
  return r >= din ? 1 : (int)((din + r - 1) / r);
}

// Smallest slice count whose workspace fits ws_bytes for a body taking the
// slice count (1 = unsliced); 0 if even the most slices allowed do not fit.
template <typename Body>
int choose_slices(const Ctx& proto, int64_t din, int64_t dout, size_t ws_bytes, Body&& body) {
  const int64_t rmul = slice_row_multiple(proto.ar, din, dout);
  for (int s = 1; s <= din; ++s) {
    const int64_t R = (din + s - 1) / s;
    if (s > 1 && (din + R - 1) / R != s) continue;  // same extent as a smaller count
    if (s > 1 && R % rmul != 0) continue;            // slices must start on whole groups
    Ctx dry = proto;
    dry.dry = true;
    dry.off = 0;
    body(dry, s);
    if (dry.off <= ws_bytes) return s;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// A (adjoint order of D)
// ---------------------------------------------------------------------------
int run_ascend(Ctx& cx, const mera_layer* L, const double* h_in, double* h_out, int placement) {
  const int64_t din = L->din, dout = L->dout;
  set_dims(cx, (int)din, (int)dout);
  LayerT t = working_layer(cx, L);
  const void* o = working_op(cx, h_in, ipow(din, 6));
  Pieces pc = build_pieces(cx, t, din, dout);
  void* Xb = cx.take_t(ipow(din, 4) * dout * dout);
  void* Z1 = cx.take_t(din * din * ipow(dout, 4));
  Bufs b = take_bufs(cx, din, dout, din);
  const double wgt = placement == MERA_AVG ? 0.5 : 1.0;
  bool first = true;
  if (placement != MERA_RIGHT) {
    cx.c(o, "pqrPQR", t.u, "PQAB", b.mid2, "pqrABR", false, wgt, 0.0);
    cx.c(b.mid2, "pqrABR", t.u, "pqab", b.mid, "rabARB", false, 1.0, 0.0);
    cx.c(b.mid, "rabARB", pc.N3, pc.n3, b.big, "rsbaADJ", false, 1.0, 0.0);
    cx.c(pc.N, "rsbdj", b.big, "rsbaADJ", Xb, "djaADJ", false, 1.0, 0.0);
    first = false;
  }
  if (placement != MERA_LEFT) {
    cx.c(o, "qrsQRS", t.u, "RSCD", b.mid2, "qrsCDQ", false, wgt, 0.0);
    cx.c(b.mid2, "qrsCDQ", t.u, "rscd", b.mid, "qcdDCQ", false, 1.0, 0.0);
    cx.c(b.mid, "qcdDCQ", pc.M3, pc.m3, b.big, "pqcdADJ", false, 1.0, 0.0);
    cx.c(pc.M, "pqcaj", b.big, "pqcdADJ", Xb, "djaADJ", false, 1.0, first ? 0.0 : 1.0);
  }
  cx.c(Xb, "djaADJ", pc.Rp, pc.rp, Z1, "ajkAJK", false, 1.0, 0.0);
  cx.c(Z1, "ajkAJK", pc.Lp, pc.lp, h_out, "ijkIJK", true, 1.0, 0.0);
  return 0;
}

// ---------------------------------------------------------------------------
// Environments: reverse mode of e = tr(h D(rho)) w.r.t. the ket copies.
// The cotangent of D[f, g] is h[g, f]: h is read with its row legs labelled as
// bra legs ("PQRpqr" for the left window).
// ---------------------------------------------------------------------------
int run_env(Ctx& cx, const mera_layer* L, const double* h_in, const double* rho_in, double* env,
            int placement, bool want_u) {
  const int64_t din = L->din, dout = L->dout;
  set_dims(cx, (int)din, (int)dout);
  LayerT t = working_layer(cx, L);
  const void* h = working_op(cx, h_in, ipow(din, 6));
  const WorkingRho rho = working_rho(cx, rho_in, dout);
  Pieces pc = build_pieces(cx, t, din, dout);
  void* X1 = cx.take_t(din * din * ipow(dout, 4));
  void* X = cx.take_t(ipow(din, 4) * dout * dout);
  Bufs b = take_bufs(cx, din, dout, din);
  void* dN = cx.take_t(ipow(din, 4) * dout);
  void* dM = cx.take_t(ipow(din, 4) * dout);
  void* dX = want_u ? nullptr : cx.take_t(ipow(din, 4) * dout * dout);
  void* V1 = want_u ? nullptr : cx.take_t(din * din * ipow(dout, 4));
  void* dLp = want_u ? nullptr : cx.take_t(din * din * dout * dout);
  void* dRp = want_u ? nullptr : cx.take_t(din * din * dout * dout);
  // env accumulators: written in FP64 directly by the final contractions
  build_x(cx, pc, rho, X1, X, true);
  const XCopies xc = want_u ? x_copies(cx, pc, X1, X, din, dout) : XCopies{X, X, "djaADJ", "djaADJ"};
  const double wgt = placement == MERA_AVG ? 0.5 : 1.0;
  bool first_env = true;
  bool first_dx = true;
  auto acc_env = [&](const void* A, const char* la, const void* B, const char* lb, const char* lc) {
    cx.c(A, la, B, lb, env, lc, true, 1.0, first_env ? 0.0 : 1.0);
    first_env = false;
  };
  if (placement != MERA_RIGHT) {
    // cotangent of the left window through the bra and ket copies of uL
    cx.c(h, "PQRpqr", t.u, "PQAB", b.mid2, "pqrABR", false, wgt, 0.0);  // G1
    if (want_u) {
      // forward Z = (N . X) . N' for the derivative of the closing ket uL
      cx.c(pc.N, "rsbdj", xc.l, xc.xl, b.big, "rsbaADJ", false, 1.0, 0.0);
      cx.c(b.big, "rsbaADJ", pc.N, "RsBDJ", b.mid, "rabABR", false, 1.0, 0.0);
      acc_env(b.mid2, "pqrABR", b.mid, "rabABR", "pqab");
    }
    cx.c(b.mid2, "pqrABR", t.u, "pqab", b.mid, "rabARB", false, 1.0, 0.0);   // G2
    cx.c(b.mid, "rabARB", pc.N3, pc.n3, b.big, "rsbaADJ", false, 1.0, 0.0);  // G3
    cx.c(b.big, "rsbaADJ", X, "djaADJ", dN, "rsbdj", false, 1.0, 0.0);        // dN
    if (want_u) {
      acc_env(dN, "rsbdj", t.w, "bcj", "rscd");  // uR inside N
    } else {
      acc_env(dN, "rsbdj", t.u, "rscd", "bcj");  // wC inside N
      cx.c(pc.N, "rsbdj", b.big, "rsbaADJ", dX, "djaADJ", false, 1.0, 0.0);
      first_dx = false;
    }
  }
  if (placement != MERA_LEFT) {
    cx.c(h, "QRSqrs", t.u, "RSCD", b.mid2, "qrsCDQ", false, wgt, 0.0);  // H1
    if (want_u) {
      cx.c(pc.M1, "qpcja", xc.r, xc.xr, b.big, "pqcdDAJ", false, 1.0, 0.0);
      cx.c(b.big, "pqcdDAJ", pc.M, "pQCAJ", b.mid, "qcdDCQ", false, 1.0, 0.0);
      acc_env(b.mid2, "qrsCDQ", b.mid, "qcdDCQ", "rscd");
    }
    cx.c(b.mid2, "qrsCDQ", t.u, "rscd", b.mid, "qcdDCQ", false, 1.0, 0.0);   // H2
    cx.c(b.mid, "qcdDCQ", pc.M3, pc.m3, b.big, "pqcdADJ", false, 1.0, 0.0);  // H3
    cx.c(b.big, "pqcdADJ", X, "djaADJ", dM, "pqcaj", false, 1.0, 0.0);        // dM
    if (want_u) {
      acc_env(dM, "pqcaj", t.w, "bcj", "pqab");  // uL inside M
    } else {
      acc_env(dM, "pqcaj", t.u, "pqab", "bcj");  // wC inside M
      cx.c(pc.M, "pqcaj", b.big, "pqcdADJ", dX, "djaADJ", false, 1.0, first_dx ? 0.0 : 1.0);
      first_dx = false;
    }
  }
  if (!want_u) {
    // isometries inside Lp and Rp (ket copies wL = w[x a i], wR = w[d y k])
    cx.c(dX, "djaADJ", pc.Rp, pc.rp, V1, "ajkAJK", false, 1.0, 0.0);
    cx.c(V1, "ajkAJK", rho.p, rho.l, dLp, "aiAI", false, 1.0, 0.0);
    acc_env(dLp, "aiAI", t.w, "xAI", "xai");
    cx.c(X1, pc.x1, dX, "djaADJ", dRp, "dkDK", false, 1.0, 0.0);
    acc_env(dRp, "dkDK", t.w, "DyK", "dyk");
  }
  return 0;
}

// ---------------------------------------------------------------------------
// checks
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Binary tree network (Fig. 1a): the layer without disentanglers.  Labels:
// fine ket a b c d, bra A B C D (din); coarse ket i j k, bra I J K (dout);
// outer legs x, y (din) traced between ket and bra; z a leg of extent 1 (outer
// products).  Left isometry w[x a i] (fine site a = its right child), centre
// w[b c j], right w[d y k] (fine site d = its left child).  The isometry whose
// lower legs are both outside the window enters through P = w^T w on its
// coarse leg, the side isometry through E[a A i I] = sum_x w[x a i] w[x A I]
// (left) or E[d D k K] = sum_y w[d y k] w[D y K] (right):
//   D_L(rho)[a b c A B C] = sum rho[i j k I J K] P[k K] E[a A i I] w[b c j] w[B C J]
//   D_R(rho)[b c d B C D] = sum rho[i j k I J K] P[i I] w[b c j] w[B C J] E[d D k K]
// Every step is at most din^6 dout multiply-adds (against din^6 dout^3 for
// the MERA cone).
// ---------------------------------------------------------------------------
struct TreeParts {
  const void* w;
  void *pr, *el, *pl, *er;  // P[k K] of the right isometry, E_L[a A i I], P[i I], E_R[d D k K]
};

TreeParts tree_parts(Ctx& cx, const double* w_d, int64_t din, int64_t dout, int placement) {
  cx.dims.set("z", 1);
  TreeParts t{};
  if (cx.ar == Arith::F64) {
    t.w = w_d;
  } else {
    void* wt = cx.take_t(din * din * dout);
    if (!cx.dry) cx.check(mera::launch_to_f32(w_d, static_cast<float*>(wt), din * din * dout,
                                              cx.ar == Arith::B3, cx.s), "to_f32(w)");
    t.w = wt;
  }
  if (placement != MERA_RIGHT) {
    t.pr = cx.take_t(dout * dout);
    t.el = cx.take_t(din * din * dout * dout);
    cx.c(t.w, "dyk", t.w, "dyK", t.pr, "kK", false, 1.0, 0.0);
    cx.c(t.w, "xai", t.w, "xAI", t.el, "aAiI", false, 1.0, 0.0);
  }
  if (placement != MERA_LEFT) {
    t.pl = cx.take_t(dout * dout);
    t.er = cx.take_t(din * din * dout * dout);
    cx.c(t.w, "xai", t.w, "xaI", t.pl, "iI", false, 1.0, 0.0);
    cx.c(t.w, "dyk", t.w, "DyK", t.er, "dDkK", false, 1.0, 0.0);
  }
  return t;
}

int run_tree_descend(Ctx& cx, int64_t din, int64_t dout, const double* w_d, const double* rho_in,
                     double* rho_out, int placement) {
  set_dims(cx, (int)din, (int)dout);
  const TreeParts t = tree_parts(cx, w_d, din, dout, placement);
  const void* rho = working_op(cx, rho_in, ipow(dout, 6));
  void* r2 = cx.take_t(ipow(dout, 4));
  void* y1 = cx.take_t(din * din * dout * dout);
  void* y2 = cx.take_t(ipow(din, 4) * dout);
  const double wgt = placement == MERA_AVG ? 0.5 : 1.0;
  bool first = true;
  if (placement != MERA_RIGHT) {
    cx.c(rho, "ijkIJK", t.pr, "kK", r2, "ijIJ", false, 1.0, 0.0);
    cx.c(r2, "ijIJ", t.el, "aAiI", y1, "aAjJ", false, 1.0, 0.0);
    cx.c(y1, "aAjJ", t.w, "bcj", y2, "aAJbc", false, 1.0, 0.0);
    cx.c(y2, "aAJbc", t.w, "BCJ", rho_out, "abcABC", true, wgt, 0.0);
    first = false;
  }
  if (placement != MERA_LEFT) {
    cx.c(rho, "ijkIJK", t.pl, "iI", r2, "jkJK", false, 1.0, 0.0);
    cx.c(r2, "jkJK", t.er, "dDkK", y1, "dDjJ", false, 1.0, 0.0);
    cx.c(y1, "dDjJ", t.w, "bcj", y2, "dDJbc", false, 1.0, 0.0);
    cx.c(y2, "dDJbc", t.w, "BCJ", rho_out, "bcdBCD", true, wgt, first ? 0.0 : 1.0);
  }
  return 0;
}

int run_tree_ascend(Ctx& cx, int64_t din, int64_t dout, const double* w_d, const double* o_in,
                    double* o_out, int placement) {
  set_dims(cx, (int)din, (int)dout);
  const TreeParts t = tree_parts(cx, w_d, din, dout, placement);
  const void* o = working_op(cx, o_in, ipow(din, 6));
  void* v1 = cx.take_t(ipow(din, 5) * dout);
  void* v2 = cx.take_t(din * din * dout * dout);
  void* v3 = cx.take_t(ipow(dout, 4));
  const double wgt = placement == MERA_AVG ? 0.5 : 1.0;
  bool first = true;
  if (placement != MERA_RIGHT) {  // adjoint of D_L: the traced site comes back as P
    cx.c(o, "abcABC", t.w, "BCJ", v1, "abcAJ", false, 1.0, 0.0);
    cx.c(v1, "abcAJ", t.w, "bcj", v2, "aAjJ", false, 1.0, 0.0);
    cx.c(v2, "aAjJ", t.el, "aAiI", v3, "ijIJ", false, 1.0, 0.0);
    cx.c(v3, "ijIJz", t.pr, "kKz", o_out, "ijkIJK", true, wgt, 0.0);
    first = false;
  }
  if (placement != MERA_LEFT) {
    cx.c(o, "bcdBCD", t.w, "BCJ", v1, "bcdDJ", false, 1.0, 0.0);
    cx.c(v1, "bcdDJ", t.w, "bcj", v2, "dDjJ", false, 1.0, 0.0);
    cx.c(v2, "dDjJ", t.er, "dDkK", v3, "jkJK", false, 1.0, 0.0);
    cx.c(t.pl, "iIz", v3, "jkJKz", o_out, "ijkIJK", true, wgt, first ? 0.0 : 1.0);
  }
  return 0;
}

// Environment of w in the tree: the derivative of e = tr(h D_P(rho)) with
// respect to the ket copies of the left, centre and right isometries (three
// contributions per window; the isometry outside the window through P).
int run_tree_env_w(Ctx& cx, int64_t din, int64_t dout, const double* w_d, const double* h_in,
                   const double* rho_in, double* env, int placement) {
  set_dims(cx, (int)din, (int)dout);
  const TreeParts t = tree_parts(cx, w_d, din, dout, placement);
  const void* h = working_op(cx, h_in, ipow(din, 6));
  const void* rho = working_op(cx, rho_in, ipow(dout, 6));
  void* r2 = cx.take_t(ipow(dout, 4));                // R12 / R23
  void* y1 = cx.take_t(din * din * dout * dout);      // forward: R . E
  void* q1 = cx.take_t(ipow(din, 5) * dout);          // cotangent . bra centre isometry
  void* q = cx.take_t(din * din * dout * dout);       // ... . ket centre isometry
  void* ge = cx.take_t(din * din * dout * dout);      // d e / d E
  void* hc = cx.take_t(ipow(dout, 4));                // d e / d R
  void* gp = cx.take_t(dout * dout);                  // d e / d P
  const double wgt = placement == MERA_AVG ? 0.5 : 1.0;
  bool first = true;
  auto acc = [&](const void* A, const char* la, const void* B, const char* lb, const char* lc) {
    cx.c(A, la, B, lb, env, lc, true, wgt, first ? 0.0 : 1.0);
    first = false;
  };
  if (placement != MERA_RIGHT) {
    cx.c(rho, "ijkIJK", t.pr, "kK", r2, "ijIJ", false, 1.0, 0.0);
    cx.c(r2, "ijIJ", t.el, "aAiI", y1, "aAjJ", false, 1.0, 0.0);
    cx.c(h, "ABCabc", t.w, "BCJ", q1, "abcAJ", false, 1.0, 0.0);
    cx.c(q1, "abcAJ", t.w, "bcj", q, "aAjJ", false, 1.0, 0.0);
    acc(q1, "abcAJ", y1, "aAjJ", "bcj");                                   // centre
    cx.c(q, "aAjJ", r2, "ijIJ", ge, "aAiI", false, 1.0, 0.0);
    acc(ge, "aAiI", t.w, "xAI", "xai");                                    // left (in E_L)
    cx.c(q, "aAjJ", t.el, "aAiI", hc, "ijIJ", false, 1.0, 0.0);
    cx.c(rho, "ijkIJK", hc, "ijIJ", gp, "kK", false, 1.0, 0.0);
    acc(gp, "kK", t.w, "dyK", "dyk");                                      // right (in P)
  }
  if (placement != MERA_LEFT) {
    cx.c(rho, "ijkIJK", t.pl, "iI", r2, "jkJK", false, 1.0, 0.0);
    cx.c(r2, "jkJK", t.er, "dDkK", y1, "dDjJ", false, 1.0, 0.0);
    cx.c(h, "BCDbcd", t.w, "BCJ", q1, "bcdDJ", false, 1.0, 0.0);
    cx.c(q1, "bcdDJ", t.w, "bcj", q, "dDjJ", false, 1.0, 0.0);
    acc(q1, "bcdDJ", y1, "dDjJ", "bcj");                                   // centre
    cx.c(q, "dDjJ", r2, "jkJK", ge, "dDkK", false, 1.0, 0.0);
    acc(ge, "dDkK", t.w, "DyK", "dyk");                                    // right (in E_R)
    cx.c(q, "dDjJ", t.er, "dDkK", hc, "jkJK", false, 1.0, 0.0);
    cx.c(rho, "ijkIJK", hc, "jkJK", gp, "iI", false, 1.0, 0.0);
    acc(gp, "iI", t.w, "xaI", "xai");                                      // left (in P)
  }
  return 0;
}

int check_tree(int32_t din, int32_t dout, const double* w_d) {
  if (!w_d) {
    set_err("isometry pointer is null");
    return MERA_EINVAL;
  }
  if (din < 1 || dout < 1) {
    set_err("dimensions must be positive");
    return MERA_ESHAPE;
  }
  if ((int64_t)dout > (int64_t)din * din) {
    set_err("dout > din^2: no isometry exists");
    return MERA_ESHAPE;
  }
  if (ipow(din, 6) * dout >= (int64_t(1) << 40) || ipow(dout, 6) >= (int64_t(1) << 40)) {
    set_err("layer too large");
    return MERA_ESHAPE;
  }
  return MERA_OK;
}

int check_layer(const mera_layer* L) {
  if (!L) {
    set_err("layer is null");
    return MERA_EINVAL;
  }
  if (!L->u_d || !L->w_d) {
    set_err("layer tensor pointer is null");
    return MERA_EINVAL;
  }
  if (L->din < 1 || L->dout < 1) {
    set_err("dimensions must be positive");
    return MERA_ESHAPE;
  }
  if ((int64_t)L->dout > (int64_t)L->din * L->din) {
    set_err("dout > din^2: no isometry exists");
    return MERA_ESHAPE;
  }
  if (ipow(L->din, 6) * L->dout >= (int64_t(1) << 40)) {
    set_err("layer too large");
    return MERA_ESHAPE;
  }
  return MERA_OK;
}

int check_enum(int placement, int precision) {
  if (placement < MERA_LEFT || placement > MERA_AVG) {
    set_err("placement out of range");
    return MERA_EINVAL;
  }
  if (precision < MERA_FP64 || precision > MERA_BF16X3) {
    set_err("precision out of range");
    return MERA_EINVAL;
  }
  return MERA_OK;
}

// Device address of `scratch` on the calling thread's current device, looked up
// with that device current on the first call there and kept per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_err(std::string("no usable current device: ") + hipGetErrorString(e));
    return MERA_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_err(std::string("static scratch address: ") + hipGetErrorString(e));
      return MERA_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MERA_OK;
}

// Turns per-launch profiling records (which create HIP events) off for a scope.
struct NoProfile {
  bool prev;
  NoProfile() : prev(g_prof_on) { g_prof_on = false; }
  ~NoProfile() { g_prof_on = prev; }
};

Arith arith_of(int precision) {
  return precision == MERA_FP64 ? Arith::F64 : precision == MERA_FP32 ? Arith::F32 : Arith::B3;
}

template <typename F>
int run_checked(Ctx& cx, void* ws, size_t ws_bytes, void* stream, F&& body) {
  // dry pass for the size, then the real pass
  Ctx dry = cx;
  dry.dry = true;
  dry.off = 0;
  body(dry);
  if (ws_bytes < dry.off) {
    set_err("workspace too small: need " + std::to_string(dry.off) + " bytes");
    return MERA_EWORKSPACE;
  }
  if (dry.off > 0 && !ws) {
    set_err("workspace pointer is null");
    return MERA_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(ws) % 256) {
    set_err("workspace must be 256-byte aligned");
    return MERA_EINVAL;
  }
  cx.dry = false;
  cx.base = static_cast<char*>(ws);
  cx.off = 0;
  cx.s = static_cast<hipStream_t>(stream);
  body(cx);
  if (cx.err != hipSuccess) return MERA_EDEVICE;
  return MERA_OK;
}

// Polar update by the Newton-Schulz iteration X <- X (3 I - X^T X) / 2 started
// from Y / ||Y||_F (all singular values in (0, 1]), which converges to the
// orthogonal polar factor U V^T of Y = U S V^T.
// The host reads the per-iteration changes in batches of kPolarBatch (one
// stream synchronisation per batch); iterations past convergence inside a batch
// leave the isometry unchanged up to rounding (quadratic convergence).
constexpr int kPolarMaxIter = 100;
constexpr int kPolarBatch = 4;

struct PolarWs {
  double *x, *xn, *g, *partial, *scal, *dg, *off;
};
PolarWs polar_layout(Ctx& cx, int64_t rows, int64_t cols) {
  PolarWs p;
  p.x = cx.take_d(rows * cols);
  p.xn = cx.take_d(rows * cols);
  p.g = cx.take_d(cols * cols);
  p.partial = cx.take_d(mera::kReduceBlocks);
  p.scal = cx.take_d(2 + kPolarBatch);
  p.dg = cx.take_d(cols);   // singular values: tridiagonal form of X^T Y
  p.off = cx.take_d(cols);
  return p;
}

// Host-side checks shared by the polar calls; `near` adds the shifted copy of
// env (rows * cols doubles) in front of the polar buffers.
int check_polar(const double* env_d, int64_t rows, int64_t cols, const double* out_d, const double* sv_d,
                const void* ws_d, size_t ws_bytes, bool near) {
  if (!env_d || !out_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  if (rows < 1 || cols < 1 || rows < cols || rows * cols >= (int64_t(1) << 31)) {
    set_err("polar needs rows >= cols >= 1");
    return MERA_ESHAPE;
  }
  if (sv_d && cols > mera::kSymEigMaxOrder) {
    set_err("polar: singular values are available for cols <= " + std::to_string(mera::kSymEigMaxOrder));
    return MERA_ESHAPE;
  }
  Ctx dry;
  dry.dry = true;
  if (near) dry.take_d(rows * cols);
  polar_layout(dry, rows, cols);
  if (ws_bytes < dry.off) {
    set_err("workspace too small: need " + std::to_string(dry.off) + " bytes");
    return MERA_EWORKSPACE;
  }
  if (!ws_d || reinterpret_cast<uintptr_t>(ws_d) % 256) {
    set_err("workspace null or not 256-byte aligned");
    return MERA_EINVAL;
  }
  return MERA_OK;
}

// Newton-Schulz polar iteration on the buffers of `p` (see polar_layout), then
// out = -X and, when sv_d is given, the eigenvalues of X^T Y (the singular
// values of Y, largest first).  Synchronises `s`.
int polar_run(PolarWs p, const double* env_d, int64_t rows, int64_t cols, double* out_d, double* sv_d,
              hipStream_t s) {
  LabelDims dims;
  dims.d['a'] = rows;
  dims.d['b'] = cols;
  dims.d['c'] = cols;
  const int64_t n = rows * cols;
  double host[2 + kPolarBatch];
  auto fail = [&](hipError_t e, const char* what) {
    set_err(std::string("polar ") + what + ": " + hipGetErrorString(e));
    return MERA_EDEVICE;
  };
  hipError_t e;
  if ((e = mera::launch_reduce(4, env_d, nullptr, n, p.partial, p.scal, s))) return fail(e, "norm");
  if ((e = hipMemcpyAsync(host, p.scal, sizeof(double), hipMemcpyDeviceToHost, s))) return fail(e, "copy");
  if ((e = hipStreamSynchronize(s))) return fail(e, "sync");
  if (!std::isfinite(host[0]) || host[0] <= 0.0) {
    if ((e = mera::launch_fill(out_d, 0.0, n, s))) return fail(e, "fill");
    if (sv_d && (e = mera::launch_fill(sv_d, 0.0, cols, s))) return fail(e, "fill");
    if ((e = hipStreamSynchronize(s))) return fail(e, "sync");
    set_err("polar: environment is zero or not finite");
    return MERA_ENUMERIC;
  }
  if ((e = mera::launch_scale_by_rsqrt(env_d, p.x, p.scal, n, s))) return fail(e, "scale");
  int it = 0;
  bool conv = false, bad = false;
  const double thr = 1e-13 * std::sqrt((double)cols);
  while (it < kPolarMaxIter && !conv && !bad) {
    const int batch = std::min(kPolarBatch, kPolarMaxIter - it);
    for (int b = 0; b < batch; ++b) {
      // X <- X (3 I - X^T X) / 2
      if ((e = mera::contract(Arith::F64, dims, p.x, "ab", p.x, "ac", p.g, "bc", true, 1.0, 0.0, s)))
        return fail(e, "gram");
      if ((e = mera::launch_scale(p.x, p.xn, 1.5, n, s))) return fail(e, "scale");
      if ((e = mera::contract(Arith::F64, dims, p.x, "ab", p.g, "bc", p.xn, "ac", true, -0.5, 1.0, s)))
        return fail(e, "update");
      if ((e = mera::launch_reduce(1, p.xn, p.x, n, p.partial, p.scal + 2 + b, s))) return fail(e, "diff");
      std::swap(p.x, p.xn);
    }
    if ((e = hipMemcpyAsync(host + 2, p.scal + 2, batch * sizeof(double), hipMemcpyDeviceToHost, s)))
      return fail(e, "copy");
    if ((e = hipStreamSynchronize(s))) return fail(e, "sync");
    for (int b = 0; b < batch && !conv && !bad; ++b) {
      ++it;
      if (!std::isfinite(host[2 + b])) bad = true;
      else if (std::sqrt(host[2 + b]) < thr) conv = true;
    }
  }
  // out = -X; singular values from X^T Y; then check that X reached an isometry: ||X||_F^2 = cols
  if ((e = mera::launch_scale(p.x, out_d, -1.0, n, s))) return fail(e, "out");
  if (sv_d) {
    if ((e = mera::contract(Arith::F64, dims, p.x, "ab", env_d, "ac", p.g, "bc", true, 1.0, 0.0, s)))
      return fail(e, "x^T y");
    if ((e = mera::launch_sym_eigvals_desc(p.g, cols, p.dg, p.off, sv_d, s))) return fail(e, "eigenvalues");
  }
  if ((e = mera::launch_reduce(4, p.x, nullptr, n, p.partial, p.scal + 1, s))) return fail(e, "fro");
  if ((e = hipMemcpyAsync(host, p.scal + 1, sizeof(double), hipMemcpyDeviceToHost, s)))
    return fail(e, "copy");
  if ((e = hipStreamSynchronize(s))) return fail(e, "sync");
  if (!conv || !(std::fabs(host[0] - (double)cols) < 1e-8 * (double)cols)) {
    set_err("polar: iteration did not reach an isometry (rank-deficient or non-finite environment)");
    return MERA_ENUMERIC;
  }
  return MERA_OK;
}


}  // namespace

extern "C" {

const char* mera_strerror(int status) {
  switch (status) {
    case MERA_OK: return "ok";
    case MERA_EINVAL: return "invalid argument";
    case MERA_ESHAPE: return "inconsistent shape";
    case MERA_EWORKSPACE: return "workspace too small";
    case MERA_EDEVICE: return "device (HIP) error";
    case MERA_ENUMERIC: return "numerical failure";
    case MERA_ENOTCONV: return "not converged";
    default: return "unknown status";
  }
}

const char* mera_last_error(void) { return g_last_error.c_str(); }

int mera_profile_begin(void) {
  for (auto& r : g_prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  g_prof_on = true;
  return MERA_OK;
}

int mera_profile_end(mera_profile_entry* out, int32_t max_entries, int32_t* n_out) {
  g_prof_on = false;
  int rc = MERA_OK;
  int32_t n = 0;
  for (auto& r : g_prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      set_err("profile event query failed");
      rc = MERA_EDEVICE;
    }
    if (out && n < max_entries) {
      std::memset(out[n].step, 0, sizeof(out[n].step));
      std::strncpy(out[n].step, r.step.c_str(), sizeof(out[n].step) - 1);
      out[n].arith = r.arith;
      out[n].op = r.op;
      out[n].flops = r.flops;
      out[n].ms = ms;
      ++n;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  if (n_out) *n_out = n;
  return rc;
}

int mera_contract(const char* la, const double* a_d, const char* lb, const double* b_d, const char* lc,
                  double* c_d, const char* labels, const int64_t* sizes, double alpha, double beta,
                  int precision, void* ws_d, size_t ws_bytes, void* hip_stream) {
  if (!la || !lb || !lc || !labels || !sizes || !a_d || !b_d || !c_d) {
    set_err("mera_contract: null argument");
    return MERA_EINVAL;
  }
  if (precision < MERA_FP64 || precision > MERA_BF16X3) {
    set_err("mera_contract: precision out of range");
    return MERA_EINVAL;
  }
  // labels: distinct printable characters with sizes >= 1
  LabelDims dims;
  std::string seen;
  for (const char* q = labels; *q; ++q) {
    const unsigned char ch = (unsigned char)*q;
    if (ch < 33 || ch > 126 || seen.find((char)ch) != std::string::npos || sizes[q - labels] < 1 ||
        sizes[q - labels] > (int64_t)1 << 30) {
      set_err("mera_contract: labels must be distinct printable characters with sizes in [1, 2^30]");
      return MERA_ESHAPE;
    }
    seen.push_back((char)ch);
    dims.d[ch] = sizes[q - labels];
  }
  const std::string sa(la), sb(lb), sc(lc);
  auto has = [](const std::string& s, char ch) { return s.find(ch) != std::string::npos; };
  auto count_of = [&](const std::string& s) -> int64_t {
    int64_t n = 1;
    for (char ch : s) n *= dims.d[(unsigned char)ch];
    return n;
  };
  // every leg known and not repeated; each output leg in exactly one operand; summed legs in both
  for (const std::string* s : {&sa, &sb, &sc}) {
    if (s->empty() || s->size() > 6) {
      set_err("mera_contract: each operand needs 1..6 legs");
      return MERA_ESHAPE;
    }
    for (size_t i = 0; i < s->size(); ++i)
      if (!has(seen, (*s)[i]) || s->find((*s)[i], i + 1) != std::string::npos) {
        set_err("mera_contract: unknown or repeated leg label");
        return MERA_ESHAPE;
      }
  }
  int64_t M = 1, N = 1, K = 1;
  for (char ch : sc) {
    if (has(sa, ch) == has(sb, ch)) {
      set_err("mera_contract: an output leg must come from exactly one operand");
      return MERA_ESHAPE;
    }
    (has(sa, ch) ? M : N) *= dims.d[(unsigned char)ch];
  }
  for (char ch : sa)
    if (!has(sc, ch)) {
      if (!has(sb, ch)) {
        set_err("mera_contract: a summed leg must appear in both operands");
        return MERA_ESHAPE;
      }
      K *= dims.d[(unsigned char)ch];
    }
  for (char ch : sb)
    if (!has(sc, ch) && !has(sa, ch)) {
      set_err("mera_contract: a summed leg must appear in both operands");
      return MERA_ESHAPE;
    }
  if (M >= ((int64_t)1 << 31) || N >= ((int64_t)1 << 31) || K >= ((int64_t)1 << 31)) {
    set_err("mera_contract: M, N and K must each stay below 2^31");
    return MERA_ESHAPE;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  return run_checked(cx, ws_d, ws_bytes, hip_stream, [&](Ctx& c) {
    c.dims = dims;
    c.scratch_elems = (size_t)std::min<int64_t>(16 * M * N, (int64_t)1 << 24);
    c.scratch = c.take_d(c.scratch_elems);
    const void* a = working_op(c, a_d, count_of(sa));
    const void* b = working_op(c, b_d, count_of(sb));
    c.c(a, la, b, lb, c_d, lc, true, alpha, beta);
  });
}

int mera_mfma_peak(int kind, void* scratch_d, size_t scratch_bytes, double* tflops_out) {
  // 2048 workgroups x 4 waves = 8 waves per SIMD on 256 CUs; about 5 ms per launch
  constexpr int kBlocks = 2048;
  if (!tflops_out || !scratch_d || kind < 0 || kind > 2) {
    set_err("mfma peak: kind must be 0 (bf16), 1 (f32) or 2 (f64); buffers non-null");
    return MERA_EINVAL;
  }
  if (scratch_bytes < sizeof(float) * kBlocks * 256) {
    set_err("mfma peak: scratch needs 2 MiB");
    return MERA_EWORKSPACE;
  }
  const int iters = kind == 0 ? 2048 : 8192;
  float* out = static_cast<float*>(scratch_d);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = MERA_OK;
  float best = 1e30f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_err(hipGetErrorString(hipGetLastError()));
    rc = MERA_EDEVICE;
  }
  for (int rep = 0; rc == MERA_OK && rep < 4; ++rep) {  // the first launch warms the clocks up
    float ms = 0.f;
    if (hipEventRecord(e0, nullptr) != hipSuccess ||
        mera::run_mfma_peak(kind, out, kBlocks, iters, nullptr) != hipSuccess ||
        hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      set_err(hipGetErrorString(hipGetLastError()));
      rc = MERA_EDEVICE;
    } else if (rep > 0 && ms < best) {
      best = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc == MERA_OK) {
    const double flops = (double)kBlocks * 4 * iters * mera::mfma_peak_flops_per_wave_iter(kind);
    *tflops_out = flops / (best * 1e-3) / 1e12;
  }
  return rc;
}

int mera_descend(const mera_layer* layer, const double* rho_in_d, double* rho_out_d, int placement,
                 int precision, void* ws_d, size_t ws_bytes, void* hip_stream) {
  OpTag tag(MERA_OP_DESCEND);
  int st = check_layer(layer);
  if (st) return st;
  if ((st = check_enum(placement, precision))) return st;
  if (!rho_in_d || !rho_out_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  const int S = choose_slices(cx, layer->din, layer->dout, ws_bytes, [&](Ctx& c, int s) {
    run_descend(c, layer, rho_in_d, rho_out_d, placement, s);
  });
  if (S == 0) {
    set_err("workspace too small even with the chi^7 intermediates sliced");
    return MERA_EWORKSPACE;
  }
  return run_checked(cx, ws_d, ws_bytes, hip_stream,
                     [&](Ctx& c) { run_descend(c, layer, rho_in_d, rho_out_d, placement, S); });
}

int mera_descend_noalloc(const mera_layer* layer, const double* rho_in_d, double* rho_out_d,
                         int placement, int precision, void* hip_stream) {
  OpTag tag(MERA_OP_DESCEND);
  int st = check_layer(layer);
  if (st) return st;
  if ((st = check_enum(placement, precision))) return st;
  if (!rho_in_d || !rho_out_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  const int S = choose_slices(cx, layer->din, layer->dout, kNoAllocScratchBytes, [&](Ctx& c, int s) {
    run_descend(c, layer, rho_in_d, rho_out_d, placement, s);
  });
  if (S == 0) {
    set_err("descend needs more than the static scratch (" + std::to_string(MERA_NOALLOC_SCRATCH_MIB) +
            " MiB) even with the chi^7 intermediates sliced");
    return MERA_EWORKSPACE;
  }
  void* ws = nullptr;
  if ((st = scratch_of_current_device(&ws))) return st;
  NoProfile quiet;
  return run_checked(cx, ws, kNoAllocScratchBytes, hip_stream,
                     [&](Ctx& c) { run_descend(c, layer, rho_in_d, rho_out_d, placement, S); });
}

int mera_tree_descend(int32_t din, int32_t dout, const double* w_d, const double* rho_in_d,
                      double* rho_out_d, int placement, int precision, void* ws_d, size_t ws_bytes,
                      void* hip_stream) {
  OpTag tag(MERA_OP_TREE_DESCEND);
  int st = check_tree(din, dout, w_d);
  if (st) return st;
  if ((st = check_enum(placement, precision))) return st;
  if (!rho_in_d || !rho_out_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  return run_checked(cx, ws_d, ws_bytes, hip_stream, [&](Ctx& c) {
    run_tree_descend(c, din, dout, w_d, rho_in_d, rho_out_d, placement);
  });
}

int mera_tree_ascend(int32_t din, int32_t dout, const double* w_d, const double* h_in_d,
                     double* h_out_d, int placement, int precision, void* ws_d, size_t ws_bytes,
                     void* hip_stream) {
  OpTag tag(MERA_OP_TREE_ASCEND);
  int st = check_tree(din, dout, w_d);
  if (st) return st;
  if ((st = check_enum(placement, precision))) return st;
  if (!h_in_d || !h_out_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  return run_checked(cx, ws_d, ws_bytes, hip_stream, [&](Ctx& c) {
    run_tree_ascend(c, din, dout, w_d, h_in_d, h_out_d, placement);
  });
}

int mera_tree_env_w(int32_t din, int32_t dout, const double* w_d, const double* h_d,
                    const double* rho_d, double* env_w_d, int placement, int precision, void* ws_d,
                    size_t ws_bytes, void* hip_stream) {
  OpTag tag(MERA_OP_TREE_ENV_W);
  int st = check_tree(din, dout, w_d);
  if (st) return st;
  if ((st = check_enum(placement, precision))) return st;
  if (!h_d || !rho_d || !env_w_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  return run_checked(cx, ws_d, ws_bytes, hip_stream, [&](Ctx& c) {
    run_tree_env_w(c, din, dout, w_d, h_d, rho_d, env_w_d, placement);
  });
}

int mera_ascend(const mera_layer* layer, const double* h_in_d, double* h_out_d, int placement,
                int precision, void* ws_d, size_t ws_bytes, void* hip_stream) {
  OpTag tag(MERA_OP_ASCEND);
  int st = check_layer(layer);
  if (st) return st;
  if ((st = check_enum(placement, precision))) return st;
  if (!h_in_d || !h_out_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  return run_checked(cx, ws_d, ws_bytes, hip_stream,
                     [&](Ctx& c) { run_ascend(c, layer, h_in_d, h_out_d, placement); });
}

int mera_env_u(const mera_layer* layer, const double* h_d, const double* rho_d, double* env_u_d,
               int placement, int precision, void* ws_d, size_t ws_bytes, void* hip_stream) {
  OpTag tag(MERA_OP_ENV_U);
  int st = check_layer(layer);
  if (st) return st;
  if ((st = check_enum(placement, precision))) return st;
  if (!h_d || !rho_d || !env_u_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  return run_checked(cx, ws_d, ws_bytes, hip_stream, [&](Ctx& c) {
    run_env(c, layer, h_d, rho_d, env_u_d, placement, true);
  });
}

int mera_env_w(const mera_layer* layer, const double* h_d, const double* rho_d, double* env_w_d,
               int placement, int precision, void* ws_d, size_t ws_bytes, void* hip_stream) {
  OpTag tag(MERA_OP_ENV_W);
  int st = check_layer(layer);
  if (st) return st;
  if ((st = check_enum(placement, precision))) return st;
  if (!h_d || !rho_d || !env_w_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  Ctx cx;
  cx.ar = arith_of(precision);
  return run_checked(cx, ws_d, ws_bytes, hip_stream, [&](Ctx& c) {
    run_env(c, layer, h_d, rho_d, env_w_d, placement, false);
  });
}

int mera_energy(const double* h_d, const double* rho_d, int64_t n, double* e_d, void* hip_stream) {
  if (!h_d || !rho_d || !e_d) {
    set_err("null tensor pointer");
    return MERA_EINVAL;
  }
  if (n < 1 || n > (int64_t(1) << 20)) {
    set_err("matrix order out of range");
    return MERA_ESHAPE;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // one workgroup in a fixed order: needs no scratch and is bitwise reproducible
  hipError_t e = mera::launch_trace_product_small(h_d, rho_d, n, e_d, s);
  if (e != hipSuccess) {
    set_err(std::string("energy: ") + hipGetErrorString(e));
    return MERA_EDEVICE;
  }
  return MERA_OK;
}

int mera_polar_update(const double* env_d, int64_t rows, int64_t cols, double* out_d, double* sv_d,
                      void* ws_d, size_t ws_bytes, void* hip_stream) {
  int st = check_polar(env_d, rows, cols, out_d, sv_d, ws_d, ws_bytes, false);
  if (st) return st;
  Ctx cx;
  cx.dry = false;
  cx.base = static_cast<char*>(ws_d);
  cx.s = static_cast<hipStream_t>(hip_stream);
  PolarWs p = polar_layout(cx, rows, cols);
  return polar_run(p, env_d, rows, cols, out_d, sv_d, cx.s);
}

int mera_polar_update_near(const double* env_d, const double* prev_d, int64_t rows, int64_t cols,
                           double tie, double* out_d, double* sv_d, void* ws_d, size_t ws_bytes,
                           void* hip_stream) {
  if (!prev_d) {
    set_err("null previous tensor");
    return MERA_EINVAL;
  }
  if (!(tie > 0.0) || !std::isfinite(tie)) {
    set_err("tie weight must be a finite number > 0");
    return MERA_EINVAL;
  }
  int st = check_polar(env_d, rows, cols, out_d, sv_d, ws_d, ws_bytes, true);
  if (st) return st;
  Ctx cx;
  cx.dry = false;
  cx.base = static_cast<char*>(ws_d);
  cx.s = static_cast<hipStream_t>(hip_stream);
  double* shifted = cx.take_d(rows * cols);
  PolarWs p = polar_layout(cx, rows, cols);
  st = polar_run(p, env_d, rows, cols, out_d, sv_d, cx.s);
  if (st != MERA_ENUMERIC) return st;
  // rank-deficient (or zero) environment: t = tie ||env||_F / ||prev||_F, then
  // the polar factor of env - t prev
  const int64_t n = rows * cols;
  double host[2];
  hipError_t e;
  auto fail = [&](hipError_t err, const char* what) {
    set_err(std::string("polar near ") + what + ": " + hipGetErrorString(err));
    return MERA_EDEVICE;
  };
  if ((e = mera::launch_reduce(4, env_d, nullptr, n, p.partial, p.scal, cx.s))) return fail(e, "norm");
  if ((e = mera::launch_reduce(4, prev_d, nullptr, n, p.partial, p.scal + 1, cx.s))) return fail(e, "norm");
  if ((e = hipMemcpyAsync(host, p.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, cx.s))) return fail(e, "copy");
  if ((e = hipStreamSynchronize(cx.s))) return fail(e, "sync");
  if (!(host[0] > 0.0) || !std::isfinite(host[0]) || !(host[1] > 0.0) || !std::isfinite(host[1]))
    return MERA_ENUMERIC;  // a zero environment or previous tensor leaves nothing to break the tie with
  const double t = tie * std::sqrt(host[0] / host[1]);
  if ((e = hipMemcpyAsync(shifted, env_d, n * sizeof(double), hipMemcpyDeviceToDevice, cx.s)))
    return fail(e, "copy");
  if ((e = mera::launch_axpby(prev_d, shifted, -t, 1.0, n, cx.s))) return fail(e, "axpby");
  return polar_run(p, shifted, rows, cols, out_d, sv_d, cx.s);
}

int mera_fixed_point_rho(const mera_layer* si, double* rho_d, int32_t iters, double tol, int precision,
                         double* resid_d, void* ws_d, size_t ws_bytes, void* hip_stream) {
  OpTag tag(MERA_OP_FIXED_POINT);
  int st = check_layer(si);
  if (st) return st;
  if ((st = check_enum(MERA_AVG, precision))) return st;
  if (si->din != si->dout) {
    set_err("fixed point needs din == dout");
    return MERA_ESHAPE;
  }
  if (!rho_d || iters < 0 || !(tol >= 0.0) || !std::isfinite(tol)) {
    set_err("null density, negative iteration count or tolerance not a finite number >= 0");
    return MERA_EINVAL;
  }
  const int64_t d = si->din;
  const int64_t n = d * d * d;
  const int64_t nn = n * n;
  Ctx cx;
  const Arith lp = arith_of(precision);
  cx.ar = lp;
  // FP64: plain power iteration.  Reduced precision: cycles of at most
  // kRefineCycle descends in the iterative-refinement form
  //   r = D64(rho) - rho,  delta <- D_lp(delta) + r  (L-1 times, delta_1 = r),
  //   rho <- normalise(sym(rho + delta)),
  // which in exact arithmetic equals L power-iteration steps
  // (rho + sum_{k<L} D^k r = D^L rho) while the low-precision products only
  // act on the correction, so their error scales with ||delta||, not ||rho||.
  // Every FP64 descend of the current density also gives its residual
  // ||D64(rho) - rho||_F / ||rho||_F; with tol > 0 the call stops at the first
  // density whose residual is <= tol.
  constexpr int kRefineCycle = 30;
  const bool want_end_residual = resid_d != nullptr || tol > 0.0;
  int status = MERA_OK;
  int S = 1;  // slices of the chi^7 intermediates (chosen below from ws_bytes)
  auto body = [&](Ctx& c) {
    double* tmp = c.take_d(nn);
    double* r = lp != Arith::F64 ? c.take_d(nn) : nullptr;
    double* dl = lp != Arith::F64 ? c.take_d(nn) : nullptr;
    double* partial = c.take_d(mera::kReduceBlocks);
    double* scal = c.take_d(4);  // trace, ||D(rho) - rho||^2, ||rho||^2, residual
    const size_t mark = c.off;
    // one descend in arithmetic a; the descend workspace is reused every time
    auto D = [&](Arith a, const double* in, double* out) {
      c.off = mark;
      const Arith save = c.ar;
      c.ar = a;
      run_descend(c, si, in, out, MERA_AVG, S);
      c.ar = save;
    };
    if (c.dry) {  // size the workspace for both arithmetics; count one iteration
      if (iters > 0 || want_end_residual) {
        D(Arith::F64, rho_d, tmp);
        const size_t hi = c.off;
        if (lp != Arith::F64 && iters > 0) D(lp, rho_d, tmp);
        c.off = std::max(hi, c.off);
      }
      return;
    }
    // residual of the current density from d64 = D64(rho_d), into scal[3]
    auto measure = [&](const double* d64) {
      c.check(mera::launch_reduce(1, d64, rho_d, nn, partial, scal + 1, c.s), "diff");
      c.check(mera::launch_reduce(4, rho_d, nullptr, nn, partial, scal + 2, c.s), "norm");
      c.check(mera::launch_sqrt_ratio(scal + 1, scal + 2, scal + 3, c.s), "ratio");
    };
    // host read of the residual (synchronises); false on a device error or NaN
    auto meets_tol = [&]() {
      double h = NAN;
      c.check(hipMemcpyAsync(&h, scal + 3, sizeof(double), hipMemcpyDeviceToHost, c.s), "copy");
      c.check(hipStreamSynchronize(c.s), "sync");
      return c.err == hipSuccess && h <= tol;
    };
    // rho <- (next + next^T) / tr(next), in FP64
    auto finish = [&](double* next) {
      c.check(mera::launch_reduce(2, next, nullptr, n, partial, scal, c.s), "trace");
      c.check(mera::launch_sym_normalize(next, rho_d, n, scal, c.s), "symmetrise");
    };
    bool measured = false;  // scal[3] holds the residual of rho_d as it is now
    bool met = false;
    if (lp == Arith::F64) {
      for (int it = 0; it < iters; ++it) {
        D(Arith::F64, rho_d, tmp);
        if (tol > 0.0) {
          measure(tmp);
          if (meets_tol()) {
            measured = met = true;
            break;
          }
        }
        finish(tmp);
      }
    } else {
      int done = 0;
      while (done < iters) {
        const int L = std::min(kRefineCycle, iters - done);
        D(Arith::F64, rho_d, tmp);                                          // D64(rho)
        if (tol > 0.0) {
          measure(tmp);
          if (meets_tol()) {
            measured = met = true;
            break;
          }
        }
        c.check(mera::launch_scale(tmp, r, 1.0, nn, c.s), "copy");          // r = D64(rho)
        c.check(mera::launch_axpby(rho_d, r, -1.0, 1.0, nn, c.s), "resid");  // r -= rho
        c.check(mera::launch_scale(r, dl, 1.0, nn, c.s), "copy");           // delta = r
        for (int j = 1; j < L; ++j) {
          D(lp, dl, tmp);                                                   // D_lp(delta)
          c.check(mera::launch_axpby(r, tmp, 1.0, 1.0, nn, c.s), "acc");    // + r
          std::swap(dl, tmp);
        }
        c.check(mera::launch_axpby(rho_d, dl, 1.0, 1.0, nn, c.s), "update");  // rho + delta
        done += L;
        finish(dl);
      }
    }
    if (!measured && want_end_residual) {  // residual of the density returned
      D(Arith::F64, rho_d, tmp);
      measure(tmp);
      if (tol > 0.0) met = meets_tol();
    }
    if (resid_d) c.check(mera::launch_scale(scal + 3, resid_d, 1.0, 1, c.s), "residual");
    if (tol > 0.0 && !met && c.err == hipSuccess) {
      set_err("fixed point: residual above tol after the iteration budget");
      status = MERA_ENOTCONV;
    }
  };
  S = choose_slices(cx, d, d, ws_bytes, [&](Ctx& c, int s) {
    S = s;
    body(c);
  });
  if (S == 0) {
    set_err("workspace too small even with the chi^7 intermediates sliced");
    return MERA_EWORKSPACE;
  }
  const int rc = run_checked(cx, ws_d, ws_bytes, hip_stream, body);
  return rc != MERA_OK ? rc : status;
}

int mera_tfim_hamiltonian(double field, double* h_host, double* shift_host) {
  if (!h_host || !shift_host || !std::isfinite(field)) {
    set_err("null pointer or non-finite field");
    return MERA_EINVAL;
  }
  // Pauli X and Z on one spin; kron products written out index by index.
  const double X[2][2] = {{0, 1}, {1, 0}}, Z[2][2] = {{1, 0}, {0, -1}};
  double h2[4][4];
  for (int i1 = 0; i1 < 2; ++i1)
    for (int i2 = 0; i2 < 2; ++i2)
      for (int j1 = 0; j1 < 2; ++j1)
        for (int j2 = 0; j2 < 2; ++j2) {
          const double d1 = i1 == j1 ? 1.0 : 0.0, d2 = i2 == j2 ? 1.0 : 0.0;
          h2[i1 * 2 + i2][j1 * 2 + j2] =
              -X[i1][j1] * X[i2][j2] - 0.5 * field * (Z[i1][j1] * d2 + d1 * Z[i2][j2]);
        }
  double h3[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      const int i12 = i >> 1, i3 = i & 1, j12 = j >> 1, j3 = j & 1;  // (s1 s2) s3
      const int i1 = i >> 2, i23 = i & 3, j1 = j >> 2, j23 = j & 3;  // s1 (s2 s3)
      h3[i][j] = 0.5 * (h2[i12][j12] * (i3 == j3 ? 1.0 : 0.0) + (i1 == j1 ? 1.0 : 0.0) * h2[i23][j23]);
    }
  // largest eigenvalue by cyclic Jacobi rotations on a copy
  double a[8][8];
  std::memcpy(a, h3, sizeof(a));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < 8; ++p)
      for (int q = p + 1; q < 8; ++q) off += a[p][q] * a[p][q];
    if (off < 1e-300) break;
    for (int p = 0; p < 8; ++p)
      for (int q = p + 1; q < 8; ++q) {
        if (std::fabs(a[p][q]) < 1e-300) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 8; ++k) {  // columns p, q
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 8; ++k) {  // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
      }
  }
  double lmax = a[0][0];
  for (int i = 1; i < 8; ++i) lmax = std::fmax(lmax, a[i][i]);
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) h_host[i * 8 + j] = h3[i][j] - (i == j ? lmax : 0.0);
  *shift_host = lmax;
  return MERA_OK;
}

size_t mera_workspace_bytes(int op, int32_t din, int32_t dout, int precision, int placement) {
  Ctx cx;
  if (precision < MERA_FP64 || precision > MERA_BF16X3) return 0;
  if (op == MERA_OP_ENERGY) return 0;
  if (op == MERA_OP_POLAR || op == MERA_OP_POLAR_NEAR) {
    if (din < 1 || dout < 1 || din < dout) return 0;
    cx.dry = true;
    if (op == MERA_OP_POLAR_NEAR) cx.take_d((int64_t)din * dout);
    polar_layout(cx, din, dout);
    return cx.off;
  }
  if (din < 1 || dout < 1 || (int64_t)dout > (int64_t)din * din) return 0;
  if (placement < MERA_LEFT || placement > MERA_AVG) return 0;
  mera_layer L{din, dout, reinterpret_cast<const double*>(256), reinterpret_cast<const double*>(256)};
  cx.ar = arith_of(precision);
  cx.dry = true;
  const double* dummy = reinterpret_cast<const double*>(256);
  double* out = reinterpret_cast<double*>(256);
  switch (op) {
    case MERA_OP_TREE_ASCEND: run_tree_ascend(cx, din, dout, dummy, dummy, out, placement); break;
    case MERA_OP_TREE_DESCEND: run_tree_descend(cx, din, dout, dummy, dummy, out, placement); break;
    case MERA_OP_TREE_ENV_W: run_tree_env_w(cx, din, dout, dummy, dummy, dummy, out, placement); break;
    case MERA_OP_ASCEND: run_ascend(cx, &L, dummy, out, placement); break;
    case MERA_OP_DESCEND: run_descend(cx, &L, dummy, out, placement); break;
    case MERA_OP_ENV_U: run_env(cx, &L, dummy, dummy, out, placement, true); break;
    case MERA_OP_ENV_W: run_env(cx, &L, dummy, dummy, out, placement, false); break;
    case MERA_OP_FIXED_POINT: {
      if (din != dout) return 0;
      const int64_t n = (int64_t)din * din * din;
      const bool refine = precision != MERA_FP64;
      cx.take_d(n * n);                  // tmp
      if (refine) {
        cx.take_d(n * n);                // r
        cx.take_d(n * n);                // delta
      }
      cx.take_d(mera::kReduceBlocks);
      cx.take_d(4);
      const size_t mark = cx.off;
      cx.ar = Arith::F64;
      run_descend(cx, &L, dummy, out, MERA_AVG);
      const size_t hi = cx.off;
      if (refine) {
        cx.off = mark;
        cx.ar = arith_of(precision);
        run_descend(cx, &L, dummy, out, MERA_AVG);
      }
      cx.off = std::max(hi, cx.off);
      break;
    }
    default: return 0;
  }
  return cx.off;
}

size_t mera_workspace_bytes_min(int op, int32_t din, int32_t dout, int precision, int placement) {
  if (op != MERA_OP_DESCEND && op != MERA_OP_FIXED_POINT)
    return mera_workspace_bytes(op, din, dout, precision, placement);
  if (precision < MERA_FP64 || precision > MERA_BF16X3) return 0;
  if (din < 1 || dout < 1 || (int64_t)dout > (int64_t)din * din) return 0;
  if (placement < MERA_LEFT || placement > MERA_AVG) return 0;
  if (op == MERA_OP_FIXED_POINT && din != dout) return 0;
  mera_layer L{din, dout, reinterpret_cast<const double*>(256), reinterpret_cast<const double*>(256)};
  const double* dummy = reinterpret_cast<const double*>(256);
  double* out = reinterpret_cast<double*>(256);
  Ctx cx;
  cx.ar = arith_of(precision);
  cx.dry = true;
  if (op == MERA_OP_DESCEND) {
    run_descend(cx, &L, dummy, out, placement, max_slices(cx.ar, din, dout));
    return cx.off;
  }
  const int64_t n = (int64_t)din * din * din;
  const bool refine = precision != MERA_FP64;
  for (int i = 0; i < (refine ? 3 : 1); ++i) cx.take_d(n * n);
  cx.take_d(mera::kReduceBlocks);
  cx.take_d(4);
  const size_t mark = cx.off;
  cx.ar = Arith::F64;
  // the FP64 and reduced-precision descends of the fixed point share one slice count
  const int S = max_slices(arith_of(precision), din, din);
  run_descend(cx, &L, dummy, out, MERA_AVG, S);
  const size_t hi = cx.off;
  if (refine) {
    cx.off = mark;
    cx.ar = arith_of(precision);
    run_descend(cx, &L, dummy, out, MERA_AVG, S);
  }
  return std::max(hi, cx.off);
}

int mera_schedule_plan(int op, int32_t din, int32_t dout, int precision, int placement, char* out,
                       size_t out_bytes, size_t* needed) {
  if (precision < MERA_FP64 || precision > MERA_BF16X3 || placement < MERA_LEFT ||
      placement > MERA_AVG) {
    set_err("mera_schedule_plan: enum out of range");
    return MERA_EINVAL;
  }
  if (din < 1 || dout < 1 || (int64_t)dout > (int64_t)din * din ||
      (op == MERA_OP_FIXED_POINT && din != dout)) {
    set_err("mera_schedule_plan: bad dimensions");
    return MERA_ESHAPE;
  }
  mera_layer L{din, dout, reinterpret_cast<const double*>(256), reinterpret_cast<const double*>(256)};
  const double* dummy = reinterpret_cast<const double*>(256);
  double* o = reinterpret_cast<double*>(256);
  std::vector<std::string> plans;
  Ctx cx;
  cx.dry = true;
  cx.ar = arith_of(precision);
  cx.plans = &plans;
  switch (op) {
    case MERA_OP_TREE_ASCEND: run_tree_ascend(cx, din, dout, dummy, dummy, o, placement); break;
    case MERA_OP_TREE_DESCEND: run_tree_descend(cx, din, dout, dummy, dummy, o, placement); break;
    case MERA_OP_TREE_ENV_W: run_tree_env_w(cx, din, dout, dummy, dummy, dummy, o, placement); break;
    case MERA_OP_ASCEND: run_ascend(cx, &L, dummy, o, placement); break;
    case MERA_OP_DESCEND: run_descend(cx, &L, dummy, o, placement); break;
    case MERA_OP_ENV_U: run_env(cx, &L, dummy, dummy, o, placement, true); break;
    case MERA_OP_ENV_W: run_env(cx, &L, dummy, dummy, o, placement, false); break;
    case MERA_OP_FIXED_POINT: run_descend(cx, &L, dummy, o, MERA_AVG); break;
    default:
      set_err("mera_schedule_plan: op has no contractions");
      return MERA_EINVAL;
  }
  std::string text;
  for (const auto& ln : plans) text += ln + "\n";
  if (needed) *needed = text.size() + 1;
  if (out && out_bytes > 0) {
    const size_t n = std::min(out_bytes - 1, text.size());
    std::memcpy(out, text.data(), n);
    out[n] = 0;
  }
  return MERA_OK;
}

double mera_flops(int op, int32_t din, int32_t dout, int placement) {
  if (din < 1 || dout < 1 || (int64_t)dout > (int64_t)din * din) return 0.0;
  if (placement < MERA_LEFT || placement > MERA_AVG) return 0.0;
  mera_layer L{din, dout, reinterpret_cast<const double*>(256), reinterpret_cast<const double*>(256)};
  Ctx cx;
  cx.dry = true;
  const double* dummy = reinterpret_cast<const double*>(256);
  double* out = reinterpret_cast<double*>(256);
  switch (op) {
    case MERA_OP_TREE_ASCEND: run_tree_ascend(cx, din, dout, dummy, dummy, out, placement); break;
    case MERA_OP_TREE_DESCEND: run_tree_descend(cx, din, dout, dummy, dummy, out, placement); break;
    case MERA_OP_TREE_ENV_W: run_tree_env_w(cx, din, dout, dummy, dummy, dummy, out, placement); break;
    case MERA_OP_ASCEND: run_ascend(cx, &L, dummy, out, placement); break;
    case MERA_OP_DESCEND: run_descend(cx, &L, dummy, out, placement); break;
    case MERA_OP_ENV_U: run_env(cx, &L, dummy, dummy, out, placement, true); break;
    case MERA_OP_ENV_W: run_env(cx, &L, dummy, dummy, out, placement, false); break;
    case MERA_OP_FIXED_POINT:
      if (din != dout) return 0.0;
      run_descend(cx, &L, dummy, out, MERA_AVG);  // per iteration
      break;
    default: return 0.0;
  }
  return cx.flops;
}

}  // extern "C"
