// ht_pending.hip -- entry points declared in ht.h whose GPU implementation is
// not part of this build yet: they validate nothing and report HT_ERR_NOTSUP.
#include "ht.h"
#include <stdint.h>

extern "C" {
int ht_rhess(double *, double *, double *, double *, int64_t, int64_t, int64_t, void *) { return HT_ERR_NOTSUP; }
int ht_rhess_z(void *, void *, void *, void *, int64_t, int64_t, int64_t, void *) { return HT_ERR_NOTSUP; }
}
