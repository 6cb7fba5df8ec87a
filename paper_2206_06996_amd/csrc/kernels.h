// kernels.h -- host-side launchers of the gfx950 kernels (definitions in sparse.hip, krylov.hip,
// amg.hip).  All launchers enqueue on the given stream and do not synchronise unless stated.
#pragma once
#include "common.h"

namespace scr {

// ---------------------------------------------------------------- primitives (sparse.hip)
// out[i] = sum_{t<i} in[t] for i in [0, n]; returns out[n] (synchronises to read it).
int64_t scan_i32(const int32_t* in, int32_t* out, int64_t n, Arena& ar, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
// device-to-device copy and zero fill of `bytes` bytes by kernels (no runtime blit)
void copy_dev(void* dst, const void* src, size_t bytes, hipStream_t s);
void zero_dev(void* p, size_t bytes, hipStream_t s);
template <typename T> void fill(T* p, T v, int64_t n, hipStream_t s);
void cast_d2f(const double* a, float* b, int64_t n, hipStream_t s);
void cast_f2d(const float* a, double* b, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- sparse (sparse.hip)
template <typename T> DSell<T> sell_from_bsr(const DBsr& A, Arena& ar, hipStream_t s);
template <typename T> void sell_free(DSell<T>& A, Arena& ar);
// Block CSR with values in T (row-wave kernels for wide rows, e.g. restriction)
template <typename T>
struct DBsrT {
    int64_t nr = 0, nc = 0;
    int br = 0, bc = 0;
    int64_t nnzb = 0;
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    T* v = nullptr;
};
template <typename T> DBsrT<T> bsrt_from_bsr(const DBsr& A, Arena& ar, hipStream_t s);

// y = A x (mode 0), y = b - A x (mode 1), y += A x (mode 2), y -= A x (mode 3)
template <typename T> void sell_mv(const DSell<T>& A, const T* x, const T* b, T* y, int mode, hipStream_t s);
// Same for the 4x4 FP64 system matrix on split vectors [v (3n); p (n)]
void sell_mv_split4(const DSell<double>& K, const double* x, const double* b, double* y, int mode, hipStream_t s);
// y = R x with a row-wave kernel (rows of R are long)
template <typename T> void bsrt_mv(const DBsrT<T>& R, const T* x, T* y, hipStream_t s);
// One smoothing step on block rows of size bs:  dn = c1*d + c2*Dinv (b - A xin);  xout = xin + dn
// (d is read when read_d, written when write_d).  zero_in: xin = 0 (no SpMV; xout = dn).
// e0/e1 (optional): events recorded by the kernel's own dispatch packet (kernel time only).
template <typename T>
void smooth_step(const DSell<T>& A, const T* Dinv, const T* b, const T* xin, T* d, T* xout, double c1,
                 double c2, bool read_d, bool write_d, bool zero_in, hipStream_t s, hipEvent_t e0 = nullptr,
                 hipEvent_t e1 = nullptr);
// x = M b for a dense row-major n x n FP64 matrix M (coarsest-level inverse)
template <typename T> void dense_mv(int64_t n, const double* M, const T* b, T* x, hipStream_t s);
// The same four operations for 1x1 matrices on three node-interleaved columns (entry 3 i + c), one
// pass over the matrix; per column bitwise the one-column result
template <typename T> void sell_mv3(const DSell<T>& A, const T* x, const T* b, T* y, int mode, hipStream_t s);
template <typename T> void bsrt_mv3(const DBsrT<T>& R, const T* x, T* y, hipStream_t s);
template <typename T>
void smooth_step3(const DSell<T>& A, const T* Dinv, const T* b, const T* xin, T* d, T* xout, double c1, double c2,
                  bool read_d, bool write_d, bool zero_in, hipStream_t s);
template <typename T> void dense_mv3(int64_t n, const double* M, const T* b, T* x, hipStream_t s);
// validate a square BSR (device); returns error bits (synchronises)
int validate_bsr(int64_t nr, int bs, int64_t nnzb, const int32_t* rp, const int32_t* ci, const double* v,
                 Arena& ar, hipStream_t s);

// ---------------------------------------------------------------- operator forms (assemble.hip)
// The linear(ised) semi-discrete residual of the unified continuum (Sec. 3.1, 3.2 at rest, 3.5) is
//   R = K_rate (v_dot, p_dot) + K_state (v, p) + K_disp (u_solid, 0) - rho M (f, 0),
// evaluated at the generalized-alpha intermediate states, and the corrector tangent divided by
// alpha_f gamma dt is c_t K_rate + K_state + K_disp / c_t (c_t = alpha_m / (alpha_f gamma dt)).
// FORM_TANGENT assembles the latter (what scr_assemble_tangent gives); the three parts have the
// rows and columns of Dirichlet dofs zeroed (zero diagonal).
enum OperatorForm { FORM_TANGENT = 0, FORM_RATE = 1, FORM_STATE = 2, FORM_DISP = 3 };
// values of one form on the assembler's pattern at time step dt (its other constants unchanged);
// u: advective velocity (n_brows x 3) for FORM_TANGENT, or NULL
void assemble_form(scr_assembler* a, int form, double dt, const double* u, double* val, hipStream_t s);
// the assembler's generalized-alpha spectral radius, and a copy of its block pattern (device)
double asmb_rho_inf(const scr_assembler* a);
void asmb_pattern(const scr_assembler* a, int32_t* rp, int32_t* ci, hipStream_t s);

// ---------------------------------------------------------------- vectors (krylov.hip)
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);   // y = a x + b y
void copy_d(int64_t n, const double* x, double* y, hipStream_t s);
void interleaved_to_split(int64_t nb, const double* a, double* sv, hipStream_t s);
void split_to_interleaved(int64_t nb, const double* sv, double* a, hipStream_t s);

}  // namespace scr
