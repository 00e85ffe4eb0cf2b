/*
 * mpnn.c - oracle side of the learned coarsest-level proposal.
 * TEST INFRASTRUCTURE ONLY (see oracle.c).
 */
#include <stdint.h>

typedef struct OG OG_fwd;

int or_learned_proposal(const void* g, const int64_t* b, const void* model, int gs,
                        const int64_t* tgt, const int64_t* maxw, int8_t* part, int64_t* pw) {
  (void)g; (void)b; (void)model; (void)gs; (void)tgt; (void)maxw; (void)part; (void)pw;
  return 9; /* not available yet */
}
