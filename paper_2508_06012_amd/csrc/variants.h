// Launch shapes of the persistent advance kernel: (threads per box, atoms
// per thread, position-array stride in LDS, neighbour list in LDS, minimum
// waves per SIMD the register allocation must allow, minimum image instead of
// ghost images, Langevin integration instead of velocity Verlet, the
// embedded-atom potential instead of LJTS).
#pragma once

#define MDEOS_VARIANTS_A(X)                                                                              \
  X(256, 1, 2048, 1, 2, 0, 0, 0) X(256, 1, 2048, 0, 2, 0, 0, 0) X(512, 1, 2048, 1, 2, 0, 0, 0) X(512, 1, 2048, 0, 2, 0, 0, 0) \
  X(512, 1, 2048, 1, 4, 0, 0, 0) X(512, 1, 2048, 0, 4, 0, 0, 0) X(256, 1, 2048, 0, 4, 0, 0, 0)
#define MDEOS_VARIANTS_B(X)                                                                              \
  X(256, 1, 3072, 1, 2, 0, 0, 0) X(256, 1, 3072, 0, 2, 0, 0, 0) X(512, 1, 3072, 1, 2, 0, 0, 0) X(512, 1, 3072, 0, 2, 0, 0, 0) \
  X(512, 1, 3072, 1, 4, 0, 0, 0) X(512, 1, 3072, 0, 4, 0, 0, 0) X(512, 2, 3072, 0, 2, 0, 0, 0) X(512, 2, 3072, 1, 2, 0, 0, 0)
#define MDEOS_VARIANTS_C(X)                                                                              \
  X(256, 1, 4096, 1, 2, 0, 0, 0) X(256, 1, 4096, 0, 2, 0, 0, 0) X(512, 1, 4096, 1, 2, 0, 0, 0) X(512, 1, 4096, 0, 2, 0, 0, 0) \
  X(512, 1, 4096, 1, 4, 0, 0, 0) X(512, 1, 4096, 0, 4, 0, 0, 0) X(512, 2, 4096, 1, 2, 0, 0, 0) X(512, 2, 4096, 0, 2, 0, 0, 0) \
  X(512, 4, 4096, 0, 2, 0, 0, 0)
#define MDEOS_VARIANTS_D(X)                                                                              \
  X(256, 1, 8176, 0, 2, 0, 0, 0) X(512, 1, 8176, 1, 2, 0, 0, 0) X(512, 1, 8176, 0, 2, 0, 0, 0) X(512, 2, 8176, 1, 2, 0, 0, 0) \
  X(512, 2, 8176, 0, 2, 0, 0, 0) X(512, 4, 8176, 1, 2, 0, 0, 0) X(512, 4, 8176, 0, 2, 0, 0, 0) X(1024, 4, 8176, 0, 2, 0, 0, 0) \
  X(1024, 4, 8176, 1, 2, 0, 0, 0) X(512, 8, 8176, 0, 1, 0, 0, 0)
#define MDEOS_VARIANTS_E(X) \
  X(512, 4, 4088, 0, 2, 1, 0, 0) X(512, 8, 4088, 0, 1, 1, 0, 0) X(512, 2, 4088, 0, 2, 1, 0, 0)
// 1024-thread shapes for boxes of 600 and more atoms: 16 waves per box in the
// 128 VGPRs that four waves per SIMD allow (they spill, yet hide latency far
// better than 512-thread shapes of twice the atoms per thread)
#define MDEOS_VARIANTS_I(X) \
  X(1024, 1, 8176, 0, 4, 0, 0, 0) X(1024, 2, 8176, 0, 4, 0, 0, 0) X(1024, 1, 4096, 0, 4, 0, 0, 0) X(1024, 1, 3072, 0, 4, 0, 0, 0)
#define MDEOS_VARIANTS_J(X) X(1024, 4, 4088, 0, 4, 1, 0, 0) X(1024, 2, 4088, 0, 4, 1, 0, 0)
// Langevin (thermostatted) shapes: one per size range, lists in device memory
#define MDEOS_VARIANTS_F(X)                                                                              \
  X(512, 1, 2048, 0, 2, 0, 1, 0) X(512, 1, 3072, 0, 2, 0, 1, 0) X(512, 1, 4096, 0, 2, 0, 1, 0) X(512, 1, 8176, 0, 2, 0, 1, 0) \
  X(512, 2, 4096, 0, 2, 0, 1, 0) X(512, 2, 8176, 0, 2, 0, 1, 0) X(512, 4, 8176, 0, 2, 0, 1, 0) X(512, 8, 8176, 0, 1, 0, 1, 0) \
  X(512, 2, 4088, 0, 2, 1, 1, 0) X(512, 4, 4088, 0, 2, 1, 1, 0) X(512, 8, 4088, 0, 1, 1, 1, 0)

// Embedded-atom shapes. Its boxes hold more ghost images per atom than LJTS
// boxes of the same N (the cutoff is a larger fraction of the edge).
#define MDEOS_VARIANTS_G(X)                                                                              \
  X(256, 1, 2048, 1, 2, 0, 0, 1) X(512, 1, 2048, 0, 2, 0, 0, 1) X(512, 1, 4096, 0, 2, 0, 0, 1)             \
  X(512, 1, 4096, 0, 4, 0, 0, 1) X(512, 2, 4096, 0, 2, 0, 0, 1) X(512, 2, 8176, 0, 2, 0, 0, 1)             \
  X(512, 4, 8176, 0, 2, 0, 0, 1) X(512, 4, 4088, 0, 2, 1, 0, 1)
// Embedded-atom Langevin shapes
#define MDEOS_VARIANTS_H(X)                                                                              \
  X(512, 1, 4096, 0, 2, 0, 1, 1) X(512, 2, 8176, 0, 2, 0, 1, 1) X(512, 4, 8176, 0, 2, 0, 1, 1)
// The embedded-atom shapes for minimum-image boxes of up to 4096 atoms, each in
// a translation unit of its own: they spill, and their register allocation
// takes most of a build's time, which then runs beside the other groups.
#define MDEOS_VARIANTS_G2(X) X(512, 8, 4088, 0, 1, 1, 0, 1)
#define MDEOS_VARIANTS_H2(X) X(512, 8, 4088, 0, 1, 1, 1, 1)

#define MDEOS_VARIANTS(X)                                                                                  \
  MDEOS_VARIANTS_A(X) MDEOS_VARIANTS_B(X) MDEOS_VARIANTS_C(X) MDEOS_VARIANTS_D(X) MDEOS_VARIANTS_E(X)         \
  MDEOS_VARIANTS_F(X) MDEOS_VARIANTS_G(X) MDEOS_VARIANTS_H(X) MDEOS_VARIANTS_G2(X) MDEOS_VARIANTS_H2(X)       \
  MDEOS_VARIANTS_I(X) MDEOS_VARIANTS_J(X)
