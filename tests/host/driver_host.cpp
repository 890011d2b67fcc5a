// Host build of the device driver's state machine (csrc/driver.hpp) for the
// CPU tests: the test supplies every evaluation from the oracle, so the
// control flow of the estimator is checked without a GPU.
#include <cmath>
#include <cstdint>
#define SFLS_HD
#include "driver.hpp"

extern "C" {
int drv_sizes(int* out) {
  out[0] = (int)sizeof(sfls::DrvParams);
  out[1] = (int)sizeof(sfls::DrvState);
  out[2] = (int)sizeof(sfls::DrvArrays);
  return 3;
}
void drv_step(const sfls::DrvParams* P, sfls::DrvState* S, const sfls::DrvArrays* A) {
  sfls::Driver<sfls::SerialTeam> d(*P, *S, *A);
  d.step();
}
}
