// Routes a Dslash launch to the object compiled for its precision, Naik
// storage and epilogue (dslash.hip is built once per combination:
// HISQ_KPREC 0 = FP64, 1 = FP32, 2 = FP32 r14 Naik, 3 = FP32 r13 Naik,
// 4 = FP32 r9 Naik).
#include "hisq_internal.h"

namespace hisq {

#define HISQ_DECL(P, E, T) \
    hipError_t launch_dslash_p##P##_e##E(int nrhs, const Tile& t, const DslashArgs<T>& a, hipStream_t s, bool cm);
HISQ_DECL(0, 0, double)
HISQ_DECL(0, 1, double)
HISQ_DECL(0, 2, double)
HISQ_DECL(0, 3, double)
HISQ_DECL(1, 0, float)
HISQ_DECL(1, 1, float)
HISQ_DECL(1, 2, float)
HISQ_DECL(2, 0, float)
HISQ_DECL(2, 1, float)
HISQ_DECL(2, 2, float)
HISQ_DECL(3, 0, float)
HISQ_DECL(3, 1, float)
HISQ_DECL(3, 2, float)
HISQ_DECL(4, 0, float)
HISQ_DECL(4, 1, float)
HISQ_DECL(4, 2, float)
#undef HISQ_DECL
#define HISQ_BDECL(P, E, T) \
    hipError_t launch_dslash_batched_p##P##_e##E(const BatchTable<T>* tab, int total_blocks, int bs, hipStream_t s);
HISQ_BDECL(0, 1, double)
HISQ_BDECL(0, 2, double)
HISQ_BDECL(1, 1, float)
HISQ_BDECL(1, 2, float)
HISQ_BDECL(2, 1, float)
HISQ_BDECL(2, 2, float)
HISQ_BDECL(3, 1, float)
HISQ_BDECL(3, 2, float)
HISQ_BDECL(4, 1, float)
HISQ_BDECL(4, 2, float)
#undef HISQ_BDECL

hipError_t launch_dslash_batched_f64(int epi, const BatchTable<double>* tab, int total_blocks,
                                     int bs, hipStream_t s)
{
    if (epi == EPI_NORM) return launch_dslash_batched_p0_e1(tab, total_blocks, bs, s);
    if (epi == EPI_CG) return launch_dslash_batched_p0_e2(tab, total_blocks, bs, s);
    return hipErrorInvalidValue;
}

hipError_t launch_dslash_batched_f32(int epi, int nk, const BatchTable<float>* tab,
                                     int total_blocks, int bs, hipStream_t s)
{
    if (epi == EPI_NORM) {
        if (nk == HISQ_NAIK_R14) return launch_dslash_batched_p2_e1(tab, total_blocks, bs, s);
        if (nk == HISQ_NAIK_R13) return launch_dslash_batched_p3_e1(tab, total_blocks, bs, s);
        if (nk == HISQ_NAIK_R9) return launch_dslash_batched_p4_e1(tab, total_blocks, bs, s);
        return launch_dslash_batched_p1_e1(tab, total_blocks, bs, s);
    }
    if (epi == EPI_CG) {
        if (nk == HISQ_NAIK_R14) return launch_dslash_batched_p2_e2(tab, total_blocks, bs, s);
        if (nk == HISQ_NAIK_R13) return launch_dslash_batched_p3_e2(tab, total_blocks, bs, s);
        if (nk == HISQ_NAIK_R9) return launch_dslash_batched_p4_e2(tab, total_blocks, bs, s);
        return launch_dslash_batched_p1_e2(tab, total_blocks, bs, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_dslash_f64(int epi, int nrhs, const Tile& t, const DslashArgs<double>& a,
                             hipStream_t s, bool cm)
{
    switch (epi) {
    case EPI_PLAIN: return launch_dslash_p0_e0(nrhs, t, a, s, cm);
    case EPI_NORM: return launch_dslash_p0_e1(nrhs, t, a, s, cm);
    case EPI_CG: return launch_dslash_p0_e2(nrhs, t, a, s, cm);
    case EPI_RESID: return launch_dslash_p0_e3(nrhs, t, a, s, cm);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dslash_f32(int epi, int nk, int nrhs, const Tile& t, const DslashArgs<float>& a,
                             hipStream_t s, bool cm)
{
#define HISQ_F32_ROUTE(P)                                              \
    switch (epi) {                                                     \
    case EPI_PLAIN: return launch_dslash_p##P##_e0(nrhs, t, a, s, cm); \
    case EPI_NORM: return launch_dslash_p##P##_e1(nrhs, t, a, s, cm);  \
    case EPI_CG: return launch_dslash_p##P##_e2(nrhs, t, a, s, cm);    \
    default: return hipErrorInvalidValue;                              \
    }
    if (nk == HISQ_NAIK_R14) {
        HISQ_F32_ROUTE(2)
    }
    if (nk == HISQ_NAIK_R13) {
        HISQ_F32_ROUTE(3)
    }
    if (nk == HISQ_NAIK_R9) {
        HISQ_F32_ROUTE(4)
    }
    HISQ_F32_ROUTE(1)
#undef HISQ_F32_ROUTE
}

}  // namespace hisq
