fun f0(ipt: W ^ 2) -> W ^ 1 {
   opt[0] = opt[0] + 6;
   whl opt[0] {
      scr[3] = opt[0] + 0;
      ife ipt[0] { hlt } {
         scr[8] = 6;
         opt[0] = ipt[0] + 3; scr[0] = ipt[1] * 2;
         opt[0] = scr[3] * 6; scr[6] = scr[0] * 3;
         opt[0] = opt[0]
      }
   }
}
