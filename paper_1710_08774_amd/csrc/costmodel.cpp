// Learned cost model hook for hfav_plan (filled in with the MLP).
#include "internal.h"

bool hfav_model_config(const hfav_chain *c, int family, const int dims[3], hfav_config *cfg) {
    (void)c; (void)family; (void)dims; (void)cfg;
    return false;
}
