// ht_pending.hip -- entry points declared in ht.h whose GPU implementation is
// not part of this build yet: they validate nothing and report HT_ERR_NOTSUP.
#include "ht.h"
#include <stdint.h>

extern "C" {
}
