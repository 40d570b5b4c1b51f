// Big batched products over A-hat (sketch, power iteration, projection, W = A-hat V).
#pragma once
#include "gemm.hpp"

namespace rt {

template <typename TA, typename TX, typename TY, typename Acc>
int big_cgemm(bool conjA, int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const TX* X, int64_t ldx,
              int64_t sX, TY* Y, int64_t ldy, int64_t sY, int batch, hipStream_t s) {
  return cgemm<TA, TX, TY, Acc>(conjA, false, M, N, K, A, lda, sA, X, ldx, sX, Y, ldy, sY, batch, (Acc)1, false, s);
}

}  // namespace rt
