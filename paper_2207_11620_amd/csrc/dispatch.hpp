// Compile-time dispatch over the supported model shapes: feature count F,
// padded input width KIN, MLP width W and operand precision P.  Each macro
// expands its body with the matching constexpr names in scope and returns
// hipErrorInvalidValue from the enclosing function for other values.
#pragma once

#define NGV_DISPATCH_F_KIN(F_, KIN_, ...)                                    \
  switch (F_ * 1000 + KIN_) {                                                \
    case 2032: { constexpr int F = 2, KIN = 32; __VA_ARGS__; } break;        \
    case 2064: { constexpr int F = 2, KIN = 64; __VA_ARGS__; } break;        \
    case 4032: { constexpr int F = 4, KIN = 32; __VA_ARGS__; } break;        \
    case 4064: { constexpr int F = 4, KIN = 64; __VA_ARGS__; } break;        \
    case 8032: { constexpr int F = 8, KIN = 32; __VA_ARGS__; } break;        \
    case 8064: { constexpr int F = 8, KIN = 64; __VA_ARGS__; } break;        \
    default: return hipErrorInvalidValue;                                    \
  }
#define NGV_DISPATCH_W(W_, ...)                                              \
  switch (W_) {                                                              \
    case 32: { constexpr int W = 32; __VA_ARGS__; } break;                   \
    case 64: { constexpr int W = 64; __VA_ARGS__; } break;                   \
    default: return hipErrorInvalidValue;                                    \
  }
#define NGV_DISPATCH_P(P_, ...)                                              \
  switch (P_) {                                                              \
    case 0: { constexpr int P = 0; __VA_ARGS__; } break;                     \
    case 1: { constexpr int P = 1; __VA_ARGS__; } break;                     \
    case 2: { constexpr int P = 2; __VA_ARGS__; } break;                     \
    default: return hipErrorInvalidValue;                                    \
  }
#define NGV_DISPATCH_KIN(KIN_, ...)                                          \
  switch (KIN_) {                                                            \
    case 32: { constexpr int KIN = 32; __VA_ARGS__; } break;                 \
    case 64: { constexpr int KIN = 64; __VA_ARGS__; } break;                 \
    default: return hipErrorInvalidValue;                                    \
  }

// Translation units built once per (precision, MLP width) define NGV_PSEL
// (0, 1 or 2) and NGV_WSEL (32 or 64); NGV_PRIMARY marks the one object of
// such a unit that also holds its shape-independent code.
#ifndef NGV_PSEL
#define NGV_PSEL 0
#endif
#ifndef NGV_WSEL
#define NGV_WSEL 32
#endif
#define NGV_PRIMARY (NGV_PSEL == 0 && NGV_WSEL == 32)
