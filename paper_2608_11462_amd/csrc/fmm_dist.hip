// Distance-kernel FMM for odd k: not built yet; odd k is rejected at plan time.
#include "phs_internal.h"
namespace phs {
void build_cheb_tables(ChebTables &t, int Q) { t.Q = Q; }
void free_cheb_tables(ChebTables &t) { t = ChebTables(); }
size_t cheb_expansion_bytes(int, int, int, bool) { return 16; }
void dist_matvec(Plan &, const double *, double *, double *, bool, hipStream_t) {
  throw Error{PHS_ERR_INVALID_ARGUMENT, "odd k not built yet"};
}
void dist_expansions(Plan &, const double *, hipStream_t) {
  throw Error{PHS_ERR_INVALID_ARGUMENT, "odd k not built yet"};
}
void dist_eval_targets(Plan &, const double *, const double *, const double *, int64_t, double *, hipStream_t) {
  throw Error{PHS_ERR_INVALID_ARGUMENT, "odd k not built yet"};
}
}
