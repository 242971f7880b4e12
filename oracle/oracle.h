/* Plain FP64 CPU oracle (test infrastructure only).  See oracle.c. */
#ifndef DFPR_ORACLE_H
#define DFPR_ORACLE_H
#include <stdint.h>

enum { ORC_STATIC = 0, ORC_ND = 1, ORC_DF = 2, ORC_DFP = 3 };
/* Frontier measure (Section 4.2): relative rank change, rank change, change of the contribution factor. */
enum { ORC_CRIT_RELATIVE = 0, ORC_CRIT_ABSOLUTE = 1, ORC_CRIT_CONTRIB = 2 };

int64_t orc_canonical(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      int32_t* esrc, int32_t* edst);
void orc_csr(int32_t n, int64_t m, const int32_t* esrc, const int32_t* edst, int by_dst,
             int32_t* off, int32_t* idx);
int orc_apply(int32_t n, int64_t m_old, const int32_t* osrc, const int32_t* odst,
              int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
              int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst,
              int32_t* new_src, int32_t* new_dst, int64_t* m_new,
              int32_t* dm_src, int32_t* dm_dst, int64_t* n_dm,
              int32_t* dp_src, int32_t* dp_dst, int64_t* n_dp, int64_t* info);
int orc_rank(int32_t n, int32_t mode,
             const int32_t* prev_off, const int32_t* prev_idx,
             const int32_t* out_off, const int32_t* out_idx,
             const int32_t* in_off, const int32_t* in_idx,
             int64_t n_dm, const int32_t* dm_src, const int32_t* dm_dst,
             int64_t n_dp, const int32_t* dp_src, const int32_t* dp_dst,
             const double* r_prev, double alpha, double tol, double tol_f, double tol_p,
             int32_t criterion, int32_t max_iters, double* r_out, int64_t* stats, double* last_delta,
             int32_t* frontier);
int orc_num_threads(void);

#endif
