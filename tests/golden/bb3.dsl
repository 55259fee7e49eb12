fun f0(ipt: W ^ 3) -> W ^ 1 {
   opt[0] = 1;
   whl opt[0] {
      opt[0] = opt[0] + ipt[0];
      ife ipt[2] { hlt } {
         scr[4] = 6;
         opt[0] = opt[0] + opt[0]
      };
      scr[6] = scr[8] * 2;
      whl ipt[1] { scr[4] = 3; opt[0] = 8 };
      scr[0] = opt[0] + 9
   }
}
