// Per-query rules of the march epilogue that do not touch the decoder, kept
// free of HIP headers so that host code (and host-side tests) can use them.
#pragma once

#if defined(__HIPCC__)
#define DIST_HD __host__ __device__
#else
#define DIST_HD
#endif

namespace dist {

// Position of a query with |f| = af among a ray's K minimum-|f| records
// (Sec. 3.4, App. B.2: the K queries of smallest |f| along the ray), given the
// records' |f| in ascending order (empty records hold +infinity): the number
// of records with |f_rec| <= af, so ties keep the earlier step.  A non-finite
// af (NaN or infinity) returns K: such a query is never recorded (the ray is
// stopped by the caller), so it cannot displace a valid record.
DIST_HD inline int topk_rank(float af, const float* rec_abs, int K) {
  if (!(af <= 3.402823466e+38f)) return K;
  int pos = 0;
  for (int k = 0; k < K; ++k) pos += (rec_abs[k] <= af) ? 1 : 0;
  return pos;
}

}  // namespace dist
