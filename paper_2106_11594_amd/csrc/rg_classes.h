// Size classes of the on-chip batched kernels (rg_rk.hip: row by row, small
// streams; rg_mf.hip: blocked, larger streams) and their launcher.
#pragma once
#include "rg_internal.h"

#define RG_NUM_CLASSES 9                      // classes of FP32 streams: 0 .. 8
#define RG_CLASS_F64 RG_NUM_CLASSES           // the blocked kernel for FP64 streams
#define RG_MAX_FAMILIES (2 + RG_NUM_CLASSES)  // family 0 = generic global-state kernel, family c + 1 = class c

namespace rg {
// Class index for a stream of m regressors and capacity r_max, or -1 when the
// stream goes to the generic kernel (too large for the chip).  FP64 streams
// (dtype 1) take RG_CLASS_F64 when it holds them.
int choose_class(int m, int r_max, int dtype);
int class_rmax(int cls);
// Whether class cls keeps the dual basis in factored form (Ct = H^-1 C, with
// H^-1 = (C C^T)^-1 in FP64): the blocked kernel's variants do.
bool class_factored(int cls);
// Raise the dynamic-LDS limit of class cls's kernel to what rows_alloc needs
// (once per handle, at init).
hipError_t prepare_class(int cls, int rows_alloc);
// One launch over a.n_order streams of class cls; rows_alloc = the largest
// r_max among them (rows of Ct reserved in LDS).
template <typename T>
hipError_t launch_push_class(int cls, const PushArgs<T> &a, int rows_alloc, hipStream_t s);
// Whether class cls can hold a stream of m regressors and capacity r_max (by
// shape; RG_CLASS_F64 takes FP64 streams only, the others FP32 streams), and
// the class's shape (rank capacity, column capacity, threads).
bool class_fits(int cls, int m, int r_max);
int class_mmax(int cls);
int class_threads(int cls);
// Process-wide placement rules (see rg_set_class_rules in rg.h).
void set_class_rules(const int *m_hi, const int *r_max_hi, const int *cls, int n);
// The blocked kernel's variants (rg_mf.hip), numbered 0..5.
int mf_choose(int m, int r_max);
bool mf_fits(int v, int m, int r_max);
int mf_mmax(int v);
int mf_threads(int v);
int mf_rmax(int v);
hipError_t mf_prepare(int v, int r_max);
hipError_t mf_launch(int v, const PushArgs<float> &a, int r_max, hipStream_t s);
// Its FP64 variant (class RG_CLASS_F64).
bool mf64_fits(int m, int r_max);
int mf64_rmax();
int mf64_mmax();
int mf64_threads();
hipError_t mf64_prepare(int r_max);
hipError_t mf64_launch(const PushArgs<double> &a, int r_max, hipStream_t s);
}  // namespace rg
