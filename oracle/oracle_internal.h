/* oracle_internal.h - types shared by the oracle's C files (test infrastructure). */
#ifndef ORACLE_INTERNAL_H
#define ORACLE_INTERNAL_H
#include <stdint.h>

typedef struct {
  int32_t n;
  int32_t* xadj;
  int32_t* adj;
  int64_t* w;
  int64_t* vc; /* cost on the CPU */
  int64_t* vg; /* cost on the GPU */
} OG;

/* learned coarsest-level proposal (mpnn.c): fills part/pw, returns a status */
int or_learned_proposal(const OG* g, const int64_t* b, const void* model, int gs,
                        const int64_t* tgt, const int64_t* maxw, int8_t* part, int64_t* pw);

#endif
