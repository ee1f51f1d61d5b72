/*
 * Plain CPU oracle for exact simulation of AIG miters (test infrastructure only).
 * Header private to oracle/; the GPU path has its own, unrelated header.
 */
#ifndef ES_ORACLE_H
#define ES_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_OK 0
#define ORACLE_ERR_PARSE (-1)
#define ORACLE_ERR_UNSUPPORTED (-2)
#define ORACLE_NONE UINT64_MAX

typedef struct oracle_aig oracle_aig;

/* Parse ASCII AIGER text.  Latches or more than 64 inputs: ORACLE_ERR_UNSUPPORTED. */
int oracle_parse_aag(const char *text, size_t len, oracle_aig **out, char *err, size_t errlen);
void oracle_free(oracle_aig *g);
uint32_t oracle_num_inputs(const oracle_aig *g);
uint32_t oracle_num_outputs(const oracle_aig *g);
uint32_t oracle_num_ands(const oracle_aig *g);

/* out_words[t] bit j = value of output j at pattern ps[t] (needs <= 64 outputs). */
int oracle_eval_outputs(const oracle_aig *g, const uint64_t *ps, size_t k, uint64_t *out_words);
/* out[t] = OR of all outputs at pattern ps[t]. */
int oracle_eval_miter(const oracle_aig *g, const uint64_t *ps, size_t k, uint8_t *out);
/* Lowest p in [lo, hi) whose miter value is 1, else ORACLE_NONE.  *evaluated = patterns simulated. */
uint64_t oracle_lowest_failure(const oracle_aig *g, uint64_t lo, uint64_t hi, int threads, uint64_t *evaluated);

#ifdef __cplusplus
}
#endif
#endif
