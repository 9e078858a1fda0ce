// Dispatch of the evaluation + elimination launches over the register
// classes (the kernels are instantiated per class in eval_elim_c<N>.hip).
#include "eval_elim.hpp"

namespace snc {

#define SNC_EXTERN_CLASS(NN)                                                                                  \
  extern template int eval_elim_grid_cls<NN>(int, int);                                                      \
  extern template int eval_elim_scratch_cls<NN>(int, int);                                                   \
  extern template void launch_eval_elim_cls<NN>(const EEVariant&, uint32_t*, const PrimeC*, const ResJob*,   \
                                                const int32_t*, const int64_t*, int, int64_t, int,            \
                                                const RowDesc*, uint32_t*, uint32_t*, AbnEntry*, uint32_t,    \
                                                bool, hipStream_t);
SNC_EXTERN_CLASS(8)
SNC_EXTERN_CLASS(16)
SNC_EXTERN_CLASS(32)
SNC_EXTERN_CLASS(40)
SNC_EXTERN_CLASS(48)
SNC_EXTERN_CLASS(64)
#undef SNC_EXTERN_CLASS

static const int kClassCap[] = {8, 16, 32, 40, 48, 64};

int fast_class_of(int maxy) {
  for (int i = 0; i < (int)(sizeof(kClassCap) / sizeof(int)); ++i)
    if (maxy <= kClassCap[i]) return i;
  return -1;
}
int fast_class_cap(int cls) { return kClassCap[cls]; }

int eval_elim_grid(int cls, int wpe, int max_T) {
  switch (kClassCap[cls]) {
    case 8: return eval_elim_grid_cls<8>(wpe, max_T);
    case 16: return eval_elim_grid_cls<16>(wpe, max_T);
    case 32: return eval_elim_grid_cls<32>(wpe, max_T);
    case 40: return eval_elim_grid_cls<40>(wpe, max_T);
    case 48: return eval_elim_grid_cls<48>(wpe, max_T);
    default: return eval_elim_grid_cls<64>(wpe, max_T);
  }
}

int eval_elim_scratch(int cls, int wpe, int max_T) {
  switch (kClassCap[cls]) {
    case 8: return eval_elim_scratch_cls<8>(wpe, max_T);
    case 16: return eval_elim_scratch_cls<16>(wpe, max_T);
    case 32: return eval_elim_scratch_cls<32>(wpe, max_T);
    case 40: return eval_elim_scratch_cls<40>(wpe, max_T);
    case 48: return eval_elim_scratch_cls<48>(wpe, max_T);
    default: return eval_elim_scratch_cls<64>(wpe, max_T);
  }
}

void launch_eval_elim(int cls, const EEVariant& v, uint32_t* counter, const ResJob* jobs_d,
                      const int32_t* job_list_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                      int max_T, const RowDesc* rows_d, uint32_t* ws, uint32_t* abn_count, AbnEntry* abn_list,
                      uint32_t abn_cap, bool reduce_in, hipStream_t s) {
  const PrimeC* primes = global_crt_tables().primes;
#define SNC_EE(NN)                                                                                            \
  launch_eval_elim_cls<NN>(v, counter, primes, jobs_d, job_list_d, blk_prefix_d, njobs, nblocks, max_T, rows_d, \
                           ws, abn_count, abn_list, abn_cap, reduce_in, s)
  switch (kClassCap[cls]) {
    case 8: SNC_EE(8); break;
    case 16: SNC_EE(16); break;
    case 32: SNC_EE(32); break;
    case 40: SNC_EE(40); break;
    case 48: SNC_EE(48); break;
    default: SNC_EE(64); break;
  }
#undef SNC_EE
}

}  // namespace snc
