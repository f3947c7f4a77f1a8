/*
 * gpgomea_ops.h -- the program alphabet of gpgomea_eval.h.
 *
 * Operator numbers 0..4 follow the value row of the paper's array encoding
 * (Fig. 1: + - x / sin); 5..10 continue in the order of the operator set of
 * Tab. 2 (cos, square, sqrt, exp, log, pow).  The paper keeps the node type in
 * a separate array; here one signed byte carries type and value: a constant
 * is GPGOMEA_SYM_CONST (its value comes from the constant list), variable k is
 * GPGOMEA_SYM_VAR0 + k, and GPGOMEA_SYM_END terminates / pads a program.
 *
 * Protected semantics (the paper does not define protection; this is the
 * library's reading, with G = GPGOMEA_GUARD and clamp(t) = min(max(t,-80),80)
 * passing NaN through):
 *   DIV(a,b)  = 1 if |b| < G else a/b          SQRT(a) = sqrt(|a|)
 *   EXP(a)    = exp(clamp(a))                  LOG(a)  = 0 if |a| < G else ln|a|
 *   POW(a,b)  = 0 if |a| < G else exp(clamp(b*ln|a|))
 */
#ifndef GPGOMEA_OPS_H
#define GPGOMEA_OPS_H

#define GPGOMEA_SYM_ADD 0
#define GPGOMEA_SYM_SUB 1
#define GPGOMEA_SYM_MUL 2
#define GPGOMEA_SYM_DIV 3
#define GPGOMEA_SYM_SIN 4
#define GPGOMEA_SYM_COS 5
#define GPGOMEA_SYM_SQ 6
#define GPGOMEA_SYM_SQRT 7
#define GPGOMEA_SYM_EXP 8
#define GPGOMEA_SYM_LOG 9
#define GPGOMEA_SYM_POW 10
#define GPGOMEA_NUM_OPS 11
#define GPGOMEA_SYM_CONST 32
#define GPGOMEA_SYM_VAR0 64
#define GPGOMEA_SYM_END (-1)

/* binary32 value nearest to 1e-6 (bit pattern 0x358637BD); the same number is
 * used as the threshold in binary64 node mode */
#define GPGOMEA_GUARD 9.99999997475242708e-07
#define GPGOMEA_CLAMP 80.0

#endif /* GPGOMEA_OPS_H */
