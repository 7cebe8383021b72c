// Launchers of the sketch translation unit (internal).
#pragma once
#include "internal.h"

namespace skne {

int sketch_kstep(int prec);
int sketch_frag_bytes(int prec);
int sketch_vt(int prec);
bool sketch_sections(int prec, int k, int r, int* KSM, int* KSS);

sketchne_status degree_powers(sketchne_ctx* c, int64_t n, const int64_t* rowptr, double alpha, double* d1,
                              double* d2);
sketchne_status scale_cols(sketchne_ctx* c, int rows, int cols, double* M, const double* s);
sketchne_status scale_rows(sketchne_ctx* c, int rows, int cols, const double* M, const double* s, double* out);
sketchne_status identity(sketchne_ctx* c, int m, double* M);
sketchne_status gather_expanded(sketchne_ctx* c, int64_t n, int ntiles, int groups, int z, const int32_t* rows,
                                const float* U, int64_t ldu, int k, const double* d1, double scale, double* Gsel);
// pscale = {2^-e, 2^e, max abs R'}: the power-of-two range balance of the FP16 operands
// (e = 0 for BF16 and FP32), chosen on the device from max |R'|
sketchne_status balance(sketchne_ctx* c, int prec, int64_t count, const double* RtT, double* pscale);
sketchne_status pack_A(sketchne_ctx* c, int prec, int ntiles, int KSM, int KSS, int k, int r, const double* RtT,
                       const double* pscale, void* out);
sketchne_status pack_B(sketchne_ctx* c, int prec, int64_t n, int64_t nrows, int64_t nvt, int KSM, int KSS, int k,
                       int r, const int32_t* gather, const float* U, int64_t ldu, const double* d1, const double* pscale,
                       void* out);
sketchne_status pack_signs(sketchne_ctx* c, int ntiles, int groups, int z, const int8_t* signs, float* sgn);
sketchne_status fused_sketch(sketchne_ctx* c, int cls, int prec, int64_t nrows, int groups, int ntiles, int KSM,
                             int KSS, const void* Bpack, const void* Apack, const float* sgn, float* out,
                             int64_t ld_out, float out_scale);
sketchne_status z_reduce(sketchne_ctx* c, int l, int z, const int8_t* signs, const float* T1t, int64_t ld_t1,
                         float inv_sqrt_z, float* Z);
sketchne_status ot_q(sketchne_ctx* c, int l, int z, int hcols, const int32_t* rows, const int8_t* signs,
                     const float* Qt, int64_t n, double inv_sqrt_z, double* Bm);

// fullvisit.hip: the full-visit variant (z nonzeros per row of S and O)
int fullvisit_nct(int prec);
sketchne_status gather_rows(sketchne_ctx* c, int64_t n, int64_t npad, int k, const float* U, int64_t ldu,
                            const double* d1, double scale, double* out);
sketchne_status pack_s_full(sketchne_ctx* c, int prec, int64_t n, int64_t njt, int nct, int z, const int32_t* cols,
                            const int8_t* signs, int width, void* out);
// Z = O^T T for a row-sparse O, T held transposed (l x n, row stride ldt);
// tmax: one device word of workspace
sketchne_status fv_z(sketchne_ctx* c, int64_t n, int l, int z, const int32_t* cols, const int8_t* signs,
                     const float* Tt, int64_t ldt, unsigned* tmax, double inv_sqrt_z, float* Z);
sketchne_status dense_rows(sketchne_ctx* c, int64_t n, int width, int z, const int32_t* cols, const int8_t* signs,
                           float inv_sqrt_z, float* out);
sketchne_status fullvisit(sketchne_ctx* c, int cls, int prec, int KSM, int64_t nrows, int64_t njt, int nct_all,
                          int width, const void* Bp, const void* A1, const void* A2, float* out, int64_t ld_out,
                          float out_scale);

}  // namespace skne
