// Work descriptors shared by the host planner and the kernels.
#pragma once

#include <stdint.h>

namespace fdet {

// Matrix-free slices of the intermediate-volume variant: the hopping matrix
// by its nonzeros (q per row, row-major; padding entries have weight 0) and
// the product-form coefficients gamma_k of the degree-n Taylor polynomial,
// premultiplied by dk.
constexpr int kMaxTaylor = 8;
struct SparseOp {
  int32_t n, q;
  const int32_t* col;   // user, N*q column indices in [0, N)
  const double* val;    // user, N*q weights K_{i, col}
  double gr[kMaxTaylor], gi[kMaxTaylor];   // gamma_k dk, re and im
};

// One problem (one field configuration).
struct Prob {
  int N, Np, Nt, pad0;
  double dk;
  const double* K;      // user, N*N real symmetric
  const double* phi;    // user, Nt*N
  double* E;            // workspace, Np*Np column-major: exp(dk K)
  double* Einv;         // workspace, Np*Np: exp(-dk K)
  int32_t* status;      // user, 1 int32
  double* logdet;       // user, 2 doubles (may be null)
  double* G;            // user, N*N interleaved complex row-major (may be null)
  double* force;        // user, Nt*N (may be null)
  double* force_im;     // user, Nt*N (may be null)
  double* outE;         // user, N*N real row-major (may be null)
  double* outX;         // user UDV export (may be null)
  double* outD;
  double* outT;
  const double* op;     // user, N*N interleaved complex row-major operator A (may be null)
  double* op_trace;     // user, Nt interleaved complex: tr((1 - G~ of row t) A) (may be null)
  const SparseOp* sp;   // descriptor region: matrix-free slices instead of E (may be null)
};

enum ItemKind : int32_t {
  IK_EXPM = 0,      // E (sign +1) or Einv (sign -1) of one problem
  IK_CHAIN = 1,     // stabilised product of a range of slices
  IK_COMBINE = 2,   // UDV(o or a) <- UDV(b) x UDV(a): stabilised product of two
  IK_CLOSE = 3,     // log det (+ G) from a UDV
  IK_FORCE = 4,     // G~ at a checkpoint from the two factors a (left) and b
                    // (right) of its cyclic product, then carried forward
                    // and backward
  IK_EXPORT = 5,    // copy a UDV out in user layout
  IK_DISPLACED = 6, // G(t, t0) = sign (P + Q^{-1})^{-1} from the UDV of P (a)
                    // and the UDV of Q^{-H} (b), into `out`
};

enum ItemFlags : int32_t {
  IF_IDENTITY = 2,     // chain: start from the identity
  IF_WANT_G = 8,       // close: also form G
  IF_OUT_LOGDET = 16,  // force: write log det M (checkpoint 0 only)
  IF_OUT_G = 32,       // force: write G = G~ of row 0 (checkpoint 0 only)
  IF_EINV = 64,        // chain: slices exp(-dk K) diag(e^{i phi_t}) (the
                       // conjugate transposes of B_t^{-1}) instead of B_t
};

// A UDV triple X diag(D) T in workspace layout.
struct Udv {
  double* X;   // cmat
  double* T;   // cmat
  double* D;   // Np doubles
};

struct Item {
  int32_t kind, prob, flags, sign;
  int32_t t0, t1;       // slice rows [t0, t1), taken mod N_t (chains may wrap)
  int32_t s, pad0;      // stabilisation interval
  int32_t nb, pad1;     // force: rows t0-1, ..., t0-nb (mod N_t) carried backward
  int32_t dep0, ndep;   // single launch: the items this one waits for are
                        // deps[dep0 .. dep0 + ndep), indices into the item list
  Udv a;                // state / right operand / result
  Udv b;                // left operand (combine), right factor (force)
  Udv o;                // combine: result (X == nullptr: into a)
  double* scr;          // scratch: 4 cmats + 2*Np doubles
  double* out;          // displaced: N*N interleaved complex, row-major
};

// State of a single-launch execution of a whole plan (one persistent kernel
// whose workgroups claim items in list order).  `epoch` counts launches of
// the plan: item i is complete in the current launch once done[i] == epoch,
// so the flags never need clearing.  Zero when the descriptors are uploaded;
// the launch's first kernel advances epoch and resets next.
struct Sched {
  uint32_t epoch;
  uint32_t next;        // next item index to claim
  uint32_t pad[62];     // own 256-byte block
};

}  // namespace fdet
