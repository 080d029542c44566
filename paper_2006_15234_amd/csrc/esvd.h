// einsumsvd internals shared by the ABI entry points and the boundary code.
#pragma once
#include "internal.h"

namespace hp {

// Leg dimensions of one zip-up einsumsvd: carry V[a,x,X,b,h,H], boundary
// S[b,u,U,c], ket T[u,y,h,g,p] and bra Bra[U,Y,H,G,p] (bra dims = ket dims).
struct ZipDims {
  int64_t a = 1, x = 1, b = 1, h = 1, u = 1, c = 1, y = 1, g = 1, d = 1;
  int64_t rows() const;
  int64_t cols() const;
  int64_t v_size() const;
  int64_t s_size() const;
  int64_t t_size() const;
};

struct ZipOperands {
  const void* V = nullptr;
  const void* S = nullptr;
  const void* T = nullptr;
  const void* Bra = nullptr;
};

struct ZipWork {
  void* W1 = nullptr;
  void* W2 = nullptr;
  void* W3 = nullptr;
};

struct OrthWork {
  double* G = nullptr;
  double* Rinv = nullptr;
  double* Racc = nullptr;
  int* flags = nullptr;
};

// A X (adjoint = false, X: cols x k) or A^* X (X: rows x k) for the zip-up
// operator; Y is written as double when y_f64 (F32 applies), else in the
// apply precision.
void zip_apply(Ctx& ctx, Prec prec, const ZipDims& z, const ZipOperands& op, int batch, int64_t k,
               bool adjoint, const void* X, void* Y, bool y_f64, const ZipWork& w);

void orthogonalize(Ctx& ctx, bool cplx, double* Y, double* P, int64_t n, int64_t k, int batch,
                   const OrthWork& w);

int64_t sketch_width(int64_t m, int64_t p, int64_t rows, int64_t cols);

// Randomized einsumsvd (Alg. 4) of the zip-up operator; operands are FP64 /
// complex128 device arrays (batch-strided by their per-instance sizes).
void zip_esvd(Ctx& ctx, bool cplx, const ZipDims& z, const ZipOperands& op, int batch,
              const hpeps_esvd_opts& o, hpeps_absorb absorb, void* U, double* sigma, void* R,
              double* log_scale);

// Exact carry V[a,x,X,b,h,H] = sum_{u,U,p} L[a,u,U,b] T[u,x,1,h,p] conj(Bra[U,X,1,H,p]).
struct CarryDims {
  int64_t a = 1, u = 1, b = 1, x = 1, h = 1, d = 1;
};
void form_carry(Ctx& ctx, bool cplx, const CarryDims& cd, const void* L, const void* T,
                const void* Bra, void* V, int batch);

}  // namespace hp
