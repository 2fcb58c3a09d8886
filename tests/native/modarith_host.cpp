#include <cstdint>
#include <cstdio>
#include <random>
#define __device__
#define __forceinline__ inline
#define __host__
namespace hipstub{}
static inline uint64_t __umul64hi(uint64_t a, uint64_t b){ return (uint64_t)(((unsigned __int128)a*b)>>64); }
// the device arithmetic, compiled for the host
#define HIP_INCLUDE_HIP_HIP_RUNTIME_H
#include "modarith.h"
using namespace fl;
int main(){
  std::mt19937_64 rng(1);
  uint64_t qs[] = {(1ull<<56)-27, 1125899906826241ull, 68719403009ull, 576460752303421441ull /* < 2^60 */};
  long bad=0, tot=0;
  for (uint64_t q : qs){
    uint64_t ninv = h_neg_inv64(q);
    bool small = q < (1ull<<56);
    for(int it=0; it<200000; ++it){
      int n = 1 + rng()%16;
      Acc56 A; acc56_zero(A); Acc128 B{0,0}; unsigned __int128 ref=0;
      for(int t=0;t<n;t++){ uint64_t a = (it&1)? q-1-(rng()%3) : rng()%q, b = (it&2)? q-1 : rng()%q;
        if(small) mac56(A,a,b); mac128(B,a,b); ref += (unsigned __int128)a*b; }
      // expected: ref * 2^-64 mod q
      uint64_t rinv = h_invmod(h_powmod(2,64,q), q);
      uint64_t want = h_mulmod((uint64_t)(ref % q), rinv, q);
      uint64_t g1 = redc(B, q, ninv); tot++; if(g1!=want) bad++;
      if(small){ uint64_t g2 = redc56(A,q,ninv); tot++; if(g2!=want) bad++; }
    }
  }
  printf("checked %ld, mismatches %ld\n", tot, bad); return bad!=0;
}
